"""Statevector emulation of the paper's quantum circuit for one time step
(oracle; test infrastructure only).

Paper: Sec. 2.1.2 (amplitude encoding of P(st, sl, d_in, d_out, y, x), Eq. 3-4),
Sec. 2.1.3 (emission as the LCU I + X/2 + ZX/2 on the source qubit, Eq. 6-8),
Sec. 2.1.4 (absorption as an R_y dilation on one ancilla, Eq. 9-10), Sec. 2.1.5
(scattering: a selector ancilla between survival and redistribution, Eq. 12
and 31; the redistribution as PREP_joint -> SELECT_RPR -> PREP_joint^dagger
over a routing register that indexes the outgoing direction, Eq. 25-30; the
per-pair rotation-phase-rotation operator with the phase matrix block-encoded
on one ancilla through its eigenbasis, Eq. 18-20, and the Stokes frame
rotation as an XX+YY rotation of Q and U, Eq. 21-24), Sec. 2.1.6 (bilinear
streaming as a linear combination of integer translations with one R_y
ancilla per axis, Eq. 34-38), Sec. 2.1.7 (absorbing edges through one
"escaped" ancilla per axis) and Sec. 2.1.8 (post-selection of every ancilla on
|0> and decoding with the known normalisation).

All gates of the circuit are real (R_y, X, Z, H, and the XX+YY gate at
beta = -pi/2), so the statevector is a real float64 array.  It is held as a
tensor with one axis of length 2 per qubit; axis 0 is the most significant
bit of the flat index.  Flat-index bits from the least significant:
    x (log2 nx), y (log2 ny), d_out (q_d), d_in (q_d), sl, st0, st1,
    em0, em1 (emission LCU), abs (absorption), sel (survival/redistribution
    selector), route (q_d), pt (phase-matrix block encoding), ax, ay
    (streaming), ex, ey (escaped markers)
with q_d = ceil(log2 n); Stokes st = 2 st1 + st0 (I, Q, U, V = 0..3).  The
data registers are the low bits, so the all-ancillas-zero block is the first
2^(data bits) amplitudes.

Readings (also in the design notes):
  * The oracle's collision-matrix block of a pair is w Z / Z_11 (see phase.py),
    i.e. w R(sigma_out) (F / a) R(sigma_in) with F the reduced Rayleigh matrix
    and a = F_11.  F / a has the eigenvalues 1 + b/a, 1 - b/a (I +- Q) and c/a
    (U, V); 1 - b/a = 2 / (1 + cos^2) exceeds 1, so the phase ancilla encodes
    F / (2 a) and the redistribution branch of the selector carries weight
    2 (1 - s) against the survival weight s (s = survival factor of Eq. 11):
    the selector's post-selected block is (s I + (1 - s) M) / (2 - s).
  * Per-cell media: the absorption rotation encodes a(c) (2 - s(c)) / lambda_max
    with lambda_max = max_c (2 - s(c)), so every cell carries the same known
    factor 1 / lambda_max after the scattering block.
  * The streaming branch b of an axis applies one controlled translation by
    floor(l) + b (the base and unit translations of Eq. 36 composed), so an
    amplitude that the unit translation would bring back inside the lattice
    is not marked as escaped by the base translation.
  * Directions are padded to 2^q_d with zero amplitude and zero weight.
  * Decoding sums the post-selected amplitudes over d_in for each d_out (the
    scattered field of direction d_out is the sum over source directions).
Not covered (refused): inflow edges, 3-D lattices, tabulated matrices, phase
mixtures, dichroic absorption and the fused-Taylor form.
"""
import math

import numpy as np

from . import lbm as _lbm
from . import phase as _phase


def _log2_exact(v, what):
    q = int(v).bit_length() - 1
    if v < 1 or (1 << q) != v:
        raise ValueError("%s must be a power of two" % what)
    return q


class Layout:
    """Qubit positions (flat-index bit numbers) of every register."""

    def __init__(self, nx, ny, n):
        self.qx = _log2_exact(nx, "nx")
        self.qy = _log2_exact(ny, "ny")
        self.qd = max(1, int(math.ceil(math.log2(n)))) if n > 1 else 1
        self.nd = 1 << self.qd
        pos = 0
        self.reg = {}

        def add(name, width):
            nonlocal pos
            self.reg[name] = list(range(pos, pos + width))   # LSB first
            pos += width
        add("x", self.qx)
        add("y", self.qy)
        add("dout", self.qd)
        add("din", self.qd)
        add("sl", 1)
        add("st", 2)
        self.ndata = pos
        add("em", 2)
        add("abs", 1)
        add("sel", 1)
        add("route", self.qd)
        add("pt", 1)
        add("ax", 1)
        add("ay", 1)
        add("ex", 1)
        add("ey", 1)
        self.nq = pos

    def bit(self, name, i=0):
        return self.reg[name][i]

    def axis(self, bit):
        """Tensor axis of a flat-index bit (axis 0 = most significant)."""
        return self.nq - 1 - bit


class Emulator:
    """One-step emulation of the circuit for a 2-D problem of the oracle."""

    def __init__(self, prob):
        if prob.fused_taylor or prob.eta is not None or prob.M2 is not None:
            raise ValueError("fused Taylor, dichroic absorption and phase mixtures are not emulated")
        if any(b == _lbm.BC_INFLOW for b in prob.bc):
            raise ValueError("inflow edges are not emulated")
        self.prob = prob
        self.L = Layout(prob.nx, prob.ny, prob.n)
        self._pairs()
        self._medium()
        self.gates = 0

    # ---- operator data -------------------------------------------------------
    def _pairs(self):
        """Per ordered pair (k <- d): weight w, frame angles, eigenvalues of F/a,
        taken from the oracle's geometry and checked against its matrix."""
        p, n, nd = self.prob, self.prob.n, self.L.nd
        self.w = np.zeros((nd, nd))          # [k_out, d_in]
        self.sig_in = np.zeros((nd, nd))
        self.sig_out = np.zeros((nd, nd))
        self.lam = np.zeros((nd, nd, 4))     # eigenvalues of F/a at st after H on st0
        self.lam[:, :, :] = 0.0
        for d in range(n):
            for k in range(n):
                blk = p.M[4 * k:4 * k + 4, 4 * d:4 * d + 4]
                w = blk[0, 0]
                ct, si, so = _phase.rpr_angles(p.dirs, k, d)
                F = _phase.rayleigh_reduced(ct)
                Zt = F / F[0, 0]
                rebuilt = w * (_phase.mueller_rotation(so) @ Zt @ _phase.mueller_rotation(si))
                if np.max(np.abs(rebuilt - blk)) > 1e-12 * max(1.0, np.max(np.abs(blk))):
                    raise ValueError("collision matrix is not of the Rayleigh rotation-phase-rotation form")
                beta, gam = Zt[0, 1], Zt[2, 2]
                self.w[k, d] = w
                self.sig_in[k, d], self.sig_out[k, d] = si, so
                self.lam[k, d] = (1.0 + beta, 1.0 - beta, gam, gam)

    def _medium(self):
        p = self.prob
        al, be = p.alpha, p.beta
        a = al + be                                   # absorption factor a(c)
        s = np.where(a > 0.0, al / np.where(a > 0.0, a, 1.0), 1.0)   # survival factor s(c)
        if np.any(a < 0.0) or np.any(a > 1.0 + 1e-15) or np.any(s < 0.0):
            raise ValueError("coefficients outside the split form 0 <= alpha, beta; alpha + beta <= 1")
        lam = 2.0 - s
        self.lam_max = float(lam.max())
        self.a_abs = a * lam / self.lam_max           # encoded absorption amplitude
        self.s_surv = s
        # the source amplitude stored in the sl = 1 sector: dt J (Eq. 8)
        self.J = p.dt * p.emission_field()

    # ---- gate primitives ---------------------------------------------------------
    def _ax(self, bits):
        return [self.L.axis(b) for b in bits]

    def _u2(self, psi, tbit, table, addr_bits=(), ctrl=None):
        """Real 2x2 gate on qubit tbit; table[addr..., 2, 2] by the values of
        the address qubits (most significant first in `addr_bits` order is the
        table's axis order); ctrl: {bit: value}."""
        self._two_level(psi, {tbit: (0, 1)}, table, addr_bits, ctrl)

    def _two_level(self, psi, pair, table, addr_bits=(), ctrl=None):
        """Rotation between the basis values v0 and v1 of the qubits in `pair`
        ({bit: (v0, v1)}): (a0, a1) -> (u00 a0 + u01 a1, u10 a0 + u11 a1)."""
        self.gates += 1
        nq = self.L.nq
        ctrl = ctrl or {}
        i0 = [slice(None)] * nq
        for b, v in ctrl.items():
            i0[self.L.axis(b)] = v
        i1 = list(i0)
        for b, (v0, v1) in pair.items():
            i0[self.L.axis(b)] = v0
            i1[self.L.axis(b)] = v1
        a0 = psi[tuple(i0)]
        a1 = psi[tuple(i1)]
        rem = [ax for ax in range(nq) if isinstance(i0[ax], slice)]
        addr_ax = self._ax(addr_bits)
        table = np.asarray(table, dtype=np.float64)
        order = sorted(range(len(addr_ax)), key=lambda i: rem.index(addr_ax[i]))
        tt = table.transpose(order + [len(addr_ax), len(addr_ax) + 1])
        shape = [2 if ax in addr_ax else 1 for ax in rem]
        u = [[tt[..., r, c].reshape(shape) for c in range(2)] for r in range(2)]
        n0 = u[0][0] * a0 + u[0][1] * a1
        n1 = u[1][0] * a0 + u[1][1] * a1
        psi[tuple(i0)] = n0
        psi[tuple(i1)] = n1

    @staticmethod
    def _ry_table(theta):
        theta = np.asarray(theta, dtype=np.float64)
        c, s = np.cos(0.5 * theta), np.sin(0.5 * theta)
        return np.stack([np.stack([c, -s], -1), np.stack([s, c], -1)], -2)

    @staticmethod
    def _bits_table(values, nbits):
        """values[v] (v an nbits-bit integer) as a table indexed by the bits,
        most significant first."""
        v = np.asarray(values, dtype=np.float64)
        return v.reshape((2,) * nbits + v.shape[1:])

    def _reg_msb(self, name):
        return list(reversed(self.L.reg[name]))

    def _shift(self, psi, axis_name, esc_name, anc_name, base, periodic):
        """Permutation of the axis register: for sl = 0, direction k = d_out
        and ancilla value b the translation is by t = base[k] + b; on an
        absorbing axis a state whose target lies outside is marked escaped
        instead (X on the escape qubit), and the unmarked states translate
        modulo the register size.  Applied as a gather: out[o] = in[src(o)]."""
        self.gates += 1
        L = self.L
        N = 1 << L.nq
        flat = psi.reshape(-1)
        o = np.arange(N, dtype=np.int64)

        def field(bits):
            v = np.zeros(N, dtype=np.int64)
            for i, b in enumerate(bits):
                v |= ((o >> b) & 1) << i
            return v
        reg = L.reg[axis_name]
        size = 1 << len(reg)
        r = field(reg)
        e = (o >> L.bit(esc_name)) & 1
        k = field(L.reg["dout"])
        b = (o >> L.bit(anc_name)) & 1
        live = ((o >> L.bit("sl")) & 1) == 0
        t = np.asarray(base, dtype=np.int64)[k] + b
        # forward: e' = e ^ [r + t outside]; r' = (r + t) mod size if e' == 0
        # inverse for the output (r', e'):
        #   e' == 0: r = (r' - t) mod size, e = [r + t outside]
        #   e' == 1: r = r',               e = 1 ^ [r + t outside]
        if periodic:
            r_src = np.where(live, np.mod(r - t, size), r)
            e_src = e
        else:
            r0 = np.mod(r - t, size)
            out0 = ((r0 + t) < 0) | ((r0 + t) >= size)
            out1 = ((r + t) < 0) | ((r + t) >= size)
            r_src = np.where(live & (e == 0), r0, r)
            e_src = np.where(live, np.where(e == 0, out0.astype(np.int64), 1 ^ out1.astype(np.int64)), e)
        src = o
        for i, bb in enumerate(reg):
            src = (src & ~(1 << bb)) | (((r_src >> i) & 1) << bb)
        src = (src & ~(1 << L.bit(esc_name))) | (e_src << L.bit(esc_name))
        psi[...] = flat[src].reshape(psi.shape)

    # ---- the circuit ---------------------------------------------------------
    def encode(self, S):
        """Amplitude encoding (Eq. 4): the live field in sl = 0 and dt J in
        sl = 1, each on the diagonal d_in = d_out; returns (psi, ||phi_0||)."""
        L, p = self.L, self.prob
        data = np.zeros((4, 2, L.nd, L.nd, p.ny, p.nx))
        dd = np.arange(p.n)
        data[:, 0, dd, dd] = np.transpose(np.asarray(S, dtype=np.float64), (1, 0, 2, 3))
        data[:, 1, dd, dd] = np.transpose(self.J, (1, 0, 2, 3))
        norm = float(np.linalg.norm(data))
        psi = np.zeros((2,) * L.nq)
        flat = psi.reshape(-1)
        # data index with st = 2 st1 + st0 at the top, then sl, d_in, d_out, y, x
        flat[:1 << L.ndata] = (data / norm).reshape(-1) if norm > 0 else 0.0
        return psi, norm

    def emission(self, psi):
        """O_emis = I + X/2 + ZX/2 on sl (Eq. 7) as an LCU over (em1, em0):
        PREP |00> = sqrt(1/2)|00> + sqrt(1/4)|01> + sqrt(1/4)|10>, SELECT
        I / X / ZX, PREP^dagger; post-selected block O_emis / 2 (Eq. 8)."""
        L = self.L
        em0, em1, sl = L.bit("em", 0), L.bit("em", 1), L.bit("sl")
        t1 = 2.0 * math.acos(math.sqrt(0.75))          # P(em1 = 0) = 3/4
        t0 = 2.0 * math.acos(math.sqrt(2.0 / 3.0))     # P(em0 = 0 | em1 = 0) = 2/3
        X = np.array([[0.0, 1.0], [1.0, 0.0]])
        Z = np.array([[1.0, 0.0], [0.0, -1.0]])
        self._u2(psi, em1, self._ry_table(t1))
        self._u2(psi, em0, self._ry_table(t0), ctrl={em1: 0})
        self._u2(psi, sl, X, ctrl={em0: 1})
        self._u2(psi, sl, X, ctrl={em1: 1})
        self._u2(psi, sl, Z, ctrl={em1: 1})
        self._u2(psi, em0, self._ry_table(-t0), ctrl={em1: 0})
        self._u2(psi, em1, self._ry_table(-t1))

    def _cell_table(self, values):
        """A per-cell table [ny, nx] as a table over the y and x qubits (most
        significant first)."""
        L = self.L
        v = np.asarray(values, dtype=np.float64)
        return v.reshape((2,) * (L.qy + L.qx) + v.shape[2:]), self._reg_msb("y") + self._reg_msb("x")

    def absorption(self, psi):
        """R_y(2 arccos a) on the absorption ancilla for the live sector, the
        angle per cell (Eq. 9): post-selected block a(c) on sl = 0."""
        L = self.L
        tab, addr = self._cell_table(self._ry_table(2.0 * np.arccos(np.clip(self.a_abs, -1.0, 1.0))))
        self._u2(psi, L.bit("abs"), tab, addr, ctrl={L.bit("sl"): 0})

    def _prep_tables(self, inverse=False):
        """The R_y tree of PREP_joint over the routing register (most
        significant first), conditioned on d_in and the route bits above."""
        L = self.L
        qd, nd = L.qd, L.nd
        levels = []
        for lev in range(qd):
            nb = qd - lev            # the bit this level sets: route bit nb - 1
            th = np.zeros((nd,) + (2,) * lev)
            for d in range(nd):
                for pre in range(1 << lev):
                    lo = pre << nb
                    node = self.w[lo:lo + (1 << nb), d].sum() if d < self.prob.n else 0.0
                    left = self.w[lo:lo + (1 << (nb - 1)), d].sum() if d < self.prob.n else 0.0
                    idx = (d,) + tuple((pre >> (lev - 1 - j)) & 1 for j in range(lev))
                    th[idx] = 2.0 * math.acos(math.sqrt(min(1.0, left / node))) if node > 0 else 0.0
            tab = self._ry_table(-th if inverse else th)
            tab = tab.reshape((2,) * qd + (2,) * lev + (2, 2))
            addr = self._reg_msb("din") + [L.bit("route", qd - 1 - j) for j in range(lev)]
            levels.append((L.bit("route", nb - 1), tab, addr))
        return levels[::-1] if inverse else levels

    def scattering(self, psi):
        """Selector LCU of survival and redistribution (Eq. 12, 31) with the
        redistribution PREP_joint -> SELECT_RPR -> PREP_joint^dagger (Eq. 26-30);
        every gate acts on the live sector only."""
        L = self.L
        sl, sel = L.bit("sl"), L.bit("sel")
        live = {sl: 0}
        both = {sl: 0, sel: 1}
        s = self.s_surv
        th_sel = 2.0 * np.arctan(np.sqrt(np.where(s > 0.0, 2.0 * (1.0 - s) / np.where(s > 0.0, s, 1.0), np.inf)))
        tab, addr = self._cell_table(self._ry_table(th_sel))
        self._u2(psi, sel, tab, addr, ctrl=live)
        # PREP_joint: the weights w(k <- d_in) on the routing register
        for bit, tab, addr in self._prep_tables():
            self._u2(psi, bit, tab, addr, ctrl=both)
        # SELECT: d_out ^= d_in (clears the diagonal copy), d_out ^= route
        X = np.array([[0.0, 1.0], [1.0, 0.0]])
        for j in range(L.qd):
            self._u2(psi, L.bit("dout", j), X, ctrl={**both, L.bit("din", j): 1})
        for j in range(L.qd):
            self._u2(psi, L.bit("dout", j), X, ctrl={**both, L.bit("route", j): 1})
        # RPR of the pair (d_out, d_in): R(sigma_in), the block encoding of
        # F / (2a) through its eigenbasis (H on st0, R_y on pt by eigenvalue,
        # H), R(sigma_out); R(psi) rotates (Q, U) as in Eq. 22
        addr_pair = self._reg_msb("dout") + self._reg_msb("din")
        st0, st1, pt = L.bit("st", 0), L.bit("st", 1), L.bit("pt")
        qu = {st0: (1, 0), st1: (0, 1)}

        def rot(sig):
            c, s2 = np.cos(2.0 * sig), np.sin(2.0 * sig)
            m = np.stack([np.stack([c, s2], -1), np.stack([-s2, c], -1)], -2)
            return m.reshape((2,) * (2 * L.qd) + (2, 2))
        self._two_level(psi, qu, rot(self.sig_in), addr_pair, ctrl=both)
        r = 1.0 / math.sqrt(2.0)
        H = np.array([[r, r], [r, -r]])
        self._u2(psi, st0, H, ctrl=both)
        th = 2.0 * np.arccos(np.clip(0.5 * self.lam, -1.0, 1.0))      # [k, d, st]
        th = np.transpose(th, (2, 0, 1))                                  # [st, k, d]
        tab = self._ry_table(th).reshape((2, 2) + (2,) * (2 * L.qd) + (2, 2))
        self._u2(psi, pt, tab, [st1, st0] + addr_pair, ctrl=both)
        self._u2(psi, st0, H, ctrl=both)
        self._two_level(psi, qu, rot(self.sig_out), addr_pair, ctrl=both)
        # PREP_joint^dagger, then the selector's inverse preparation
        for bit, tab, addr in self._prep_tables(inverse=True):
            self._u2(psi, bit, tab, addr, ctrl=both)
        tab, addr = self._cell_table(self._ry_table(-th_sel))
        self._u2(psi, sel, tab, addr, ctrl=live)

    def streaming(self, psi):
        """Eq. 36-38 per axis: R_y(theta(d_out)) on the axis ancilla with
        sin^2(theta/2) = f, the translation by floor(l) + b on branch b, and
        R_y(-theta); absorbing axes mark escapes (Sec. 2.1.7)."""
        L, p = self.L, self.prob
        for ax, (name, anc, esc) in enumerate((("x", "ax", "ex"), ("y", "ay", "ey"))):
            base = np.zeros(L.nd, dtype=np.int64)
            th = np.zeros(L.nd)
            for d in range(p.n):
                l = p.shifts[d, ax]
                i0 = math.floor(l)
                f = l - i0
                base[d] = i0
                th[d] = 2.0 * math.asin(math.sqrt(f))
            periodic = p.bc[0 if ax == 0 else 2] == _lbm.BC_PERIODIC
            addr = self._reg_msb("dout")
            live = {L.bit("sl"): 0}
            self._u2(psi, L.bit(anc), self._ry_table(th).reshape((2,) * L.qd + (2, 2)), addr, ctrl=live)
            self._shift(psi, name, esc, anc, base, periodic)
            self._u2(psi, L.bit(anc), self._ry_table(-th).reshape((2,) * L.qd + (2, 2)), addr, ctrl=live)

    def post_select(self, psi):
        """Amplitudes with every ancilla |0> (Sec. 2.1.8), as
        [st, sl, d_in, d_out, y, x], and the success probability."""
        L, p = self.L, self.prob
        flat = psi.reshape(-1)[:1 << L.ndata]
        return flat.reshape(4, 2, L.nd, L.nd, p.ny, p.nx), float(np.dot(flat, flat))

    def decode(self, block, norm):
        """S'[k, st, y, x] = sum over d_in of the live amplitudes at d_out = k,
        times the known normalisation 2 lambda_max ||phi_0||."""
        S = block[:, 0].sum(axis=1)[:, :self.prob.n]        # [st, k, y, x]
        return np.transpose(S, (1, 0, 2, 3)) * (2.0 * self.lam_max * norm)

    def step(self, S):
        """One emulated step: encode, emission, absorption, scattering,
        streaming, post-select, decode.  Returns (S', success probability)."""
        psi, norm = self.encode(S)
        self.emission(psi)
        self.absorption(psi)
        self.scattering(psi)
        self.streaming(psi)
        block, p = self.post_select(psi)
        return self.decode(block, norm), p


def run(S0, prob, nsteps):
    """nsteps emulated steps, re-encoding the decoded field each step (the
    escape markers and every other ancilla start from |0> again)."""
    em = Emulator(prob)
    S = np.array(S0, dtype=np.float64)
    probs = []
    for _ in range(nsteps):
        S, p = em.step(S)
        probs.append(p)
    return S, probs
