"""Pins of the oracle's three-dimensional lattice against what does not depend
on it: the 2-D oracle (whose own pins are the paper's printed values) for
lattices that are one layer deep or uniform in z, an independent streaming
formulation with numpy's roll and zero-filled shifts, intensity conservation
on a closed lattice, and the closed form of a beam entering the top face."""
import numpy as np
import pytest

import workloads as W
from oracle import directions as OD
from oracle import lbm as OL
from oracle import lbm3d as O3


def spec3(nx=7, ny=6, nz=5, bc6=(0, 0, 0, 0, 0, 0), **kw):
    kw.setdefault("n_zen", 2)
    kw.setdefault("n_az", 4)
    return W.spec("beam3d", nx=nx, ny=ny, nz=nz, bc6=bc6, **kw)


def test_one_layer_periodic_in_z_equals_the_2d_horizontal_lattice():
    """nz = 1 with periodic z: both z taps land on the only layer and their
    weights sum to one, so the 3-D step is the 2-D step on the horizontal
    plane with l = courant (k_x, k_y)."""
    s3 = spec3(nx=9, ny=7, nz=1, bc6=(1, 1, 2, 2, 0, 0), n_zen=4, n_az=8)
    med = W.medium(s3)
    med["inflow"][2:4, :, 0] = 0.3
    p3 = O3.make_problem(s3, med)
    s2 = dict(s3, plane="xy", bc=(1, 1, 2, 2))
    med2 = dict(med, tau=med["tau"][0], albedo=med["albedo"][0], emis=med["emis"][0], inflow=med["inflow"][:4])
    p2 = OL.make_problem(s2, med2)
    S0 = W.initial_state(s3, "random")
    S3 = O3.run(S0, p3, 6)
    S2 = OL.run(S0[:, :, 0], p2, 6)
    assert np.abs(S3[:, :, 0] - S2).max() < 1e-13 * np.abs(S2).max()


def test_z_uniform_field_stays_uniform_and_follows_the_2d_lattice():
    s3 = spec3(nx=6, ny=5, nz=4, bc6=(0, 0, 1, 1, 0, 0), n_zen=4, n_az=8)
    med = W.medium(s3)
    for k in ("tau", "albedo", "emis"):
        med[k] = np.broadcast_to(med[k][:1], med[k].shape).copy()
    p3 = O3.make_problem(s3, med)
    s2 = dict(s3, plane="xy", bc=(0, 0, 1, 1))
    med2 = dict(med, tau=med["tau"][0], albedo=med["albedo"][0], emis=med["emis"][0], inflow=med["inflow"][:4])
    p2 = OL.make_problem(s2, med2)
    S2_0 = W.initial_state(dict(s3, plane="xy"), "random")
    S0 = np.broadcast_to(S2_0[:, :, None], (p3.n, 4, 4, 5, 6)).copy()
    S3 = O3.run(S0, p3, 5)
    S2 = OL.run(S2_0, p2, 5)
    for z in range(4):
        assert np.abs(S3[:, :, z] - S2).max() < 1e-13 * np.abs(S2).max()


def _shift(a, o, axis, periodic):
    """a read at index - o along axis: np.roll when periodic, else zero fill."""
    if periodic:
        return np.roll(a, o, axis=axis)
    out = np.zeros_like(a)
    n = a.shape[axis]
    if abs(o) >= n:
        return out
    src = [slice(None)] * a.ndim
    dst = [slice(None)] * a.ndim
    if o >= 0:
        src[axis], dst[axis] = slice(0, n - o), slice(o, n)
    else:
        src[axis], dst[axis] = slice(-o, n), slice(0, n + o)
    out[tuple(dst)] = a[tuple(src)]
    return out


@pytest.mark.parametrize("bc6", [(0, 0, 0, 0, 0, 0), (1, 1, 1, 1, 1, 1), (0, 0, 1, 1, 0, 0), (1, 1, 0, 0, 1, 1)])
def test_stream_equals_roll_and_zero_fill_formulation(bc6):
    s3 = spec3(nx=6, ny=5, nz=4, bc6=bc6, n_zen=4, n_az=5, az_offset_deg=10.0, courant=0.8)
    med = W.medium(s3)
    p3 = O3.make_problem(s3, med)
    rng = np.random.default_rng(2)
    Y = rng.standard_normal(p3.shape)
    got = O3.stream(Y, p3)
    ref = np.zeros_like(Y)
    for d in range(p3.n):
        lx, ly, lz = p3.shifts[d]
        for ox, wx in OL._taps(lx):
            for oy, wy in OL._taps(ly):
                for oz, wz in OL._taps(lz):
                    t = _shift(Y[d], ox, 3, bc6[0] == 0)
                    t = _shift(t, oy, 2, bc6[2] == 0)
                    t = _shift(t, oz, 1, bc6[4] == 0)
                    ref[d] += wx * wy * wz * t
    assert np.abs(got - ref).max() < 1e-14


def test_closed_lattice_conserves_intensity():
    s3 = spec3(nx=5, ny=4, nz=6, bc6=(0, 0, 0, 0, 0, 0), n_zen=4, n_az=8, renorm_irow=True)
    med = W.medium(s3)
    med["albedo"][:] = 1.0
    med["emis"][:] = 0.0
    p3 = O3.make_problem(s3, med)
    S0 = W.initial_state(s3, "random")
    S = O3.run(S0, p3, 8)
    assert S[:, 0].sum() == pytest.approx(S0[:, 0].sum(), rel=1e-12)


def test_beam_entering_the_top_face():
    """Zero field, periodic x and y, inflow on z+: after one step the top
    layer holds (1 - f_z) of the inflow for every downward direction, where
    f_z is the fractional part of its l_z, and nothing elsewhere."""
    s3 = spec3(nx=4, ny=3, nz=5, bc6=(0, 0, 0, 0, 1, 2), n_zen=4, n_az=8)
    med = W.medium(s3)
    med["inflow"][5, :, 0] = 1.0
    p3 = O3.make_problem(s3, med)
    S = O3.step(np.zeros(p3.shape), p3)
    for d in range(p3.n):
        lz = p3.shifts[d, 2]
        if lz < 0:
            fz = lz - np.floor(lz)
            assert np.allclose(S[d, 0, -1], 1.0 - fz, rtol=1e-14, atol=0)
            assert np.all(S[d, 0, :-1] == 0.0)
        else:
            assert np.all(S[d] == 0.0)
    assert np.all(S[:, 1:] == 0.0)


def test_face_validation():
    s3 = spec3(bc6=(0, 1, 0, 0, 0, 0))
    with pytest.raises(ValueError):
        O3.make_problem(s3, W.medium(s3))
    dirs = OD.make_directions(2, 4)
    with pytest.raises(ValueError):
        O3.Problem3D(4, 4, 4, dirs, 1.5, (0,) * 6, np.eye(32), 1.0, np.zeros((4, 4, 4)), np.zeros((4, 4, 4)),
                     np.zeros((4, 4, 4)), np.zeros((8, 4)))


@pytest.mark.parametrize("bc6", [(0, 0, 0, 0, 0, 0), (1, 1, 2, 1, 0, 0), (2, 2, 0, 0, 1, 2)])
def test_stream_transpose_is_the_transpose(bc6):
    """<L Y, G> = <Y, L^T G> for the linear part (inflow ghosts zeroed)."""
    s3 = spec3(nx=5, ny=4, nz=6, bc6=bc6, n_zen=4, n_az=5, az_offset_deg=10.0, courant=0.9)
    med = W.medium(s3)
    med["inflow"][:] = 0.0
    p3 = O3.make_problem(s3, med)
    rng = np.random.default_rng(8)
    Y, G = rng.standard_normal(p3.shape), rng.standard_normal(p3.shape)
    lhs = np.sum(O3.stream(Y, p3) * G)
    rhs = np.sum(Y * O3.stream_transpose(G, p3))
    assert lhs == pytest.approx(rhs, rel=1e-12)


MIXTURES = {"mixture": {"kind": "hg", "g": -0.4},
            "mixture3": [{"kind": "hg", "g": -0.4}, {"kind": "rayleigh"}]}


@pytest.mark.parametrize("ext", [None, "mixture", "mixture3", "dichroism"])
def test_adjoint3d_matches_central_differences(ext):
    s3 = spec3(nx=4, ny=3, nz=3, bc6=(1, 1, 0, 0, 1, 2), n_zen=2, n_az=4, source="uniform_emis", emis_max=0.05,
               mixture=MIXTURES.get(ext),
               dichroism=0.8 if ext == "dichroism" else None)
    med = W.medium(s3)
    med["tau"] = med["tau"] * 40.0
    p3 = O3.make_problem(s3, med)
    rng = np.random.default_rng(12)
    S0 = np.abs(rng.standard_normal(p3.shape)) * 0.1
    G = rng.standard_normal(p3.shape)
    T = 5
    res = O3.adjoint(S0, p3, T, G)

    def loss(m):
        return np.sum(O3.run(S0, O3.make_problem(s3, m), T) * G)
    for key, field in (("g_tau", "tau"), ("g_albedo", "albedo"), ("g_emis", "emis")):
        for cell in ((0, 0, 0), (1, 2, 3), (2, 1, 1)):
            h = 1e-3 * max(abs(med[field][cell]), 1e-2)   # roundoff of the O(1) loss dominates below
            mp, mm = dict(med), dict(med)
            mp[field] = med[field].copy()
            mm[field] = med[field].copy()
            mp[field][cell] += h
            mm[field][cell] -= h
            fd = (loss(mp) - loss(mm)) / (2 * h)
            assert res[key][cell] == pytest.approx(fd, rel=1e-6, abs=1e-11), (key, cell)
    # lambda0 = dLoss/dS0
    d = np.zeros(p3.shape)
    d[1, 2, 1, 0, 2] = 1e-6
    fd = (np.sum(O3.run(S0 + d, p3, T) * G) - np.sum(O3.run(S0 - d, p3, T) * G)) / 2e-6
    assert res["lambda0"][1, 2, 1, 0, 2] == pytest.approx(fd, rel=1e-6)


def test_adjoint3d_one_layer_equals_the_2d_adjoint():
    from oracle import adjoint as OA
    s3 = spec3(nx=6, ny=5, nz=1, bc6=(1, 1, 0, 0, 0, 0), n_zen=4, n_az=8)
    med = W.medium(s3)
    p3 = O3.make_problem(s3, med)
    s2 = dict(s3, plane="xy", bc=(1, 1, 0, 0))
    med2 = dict(med, tau=med["tau"][0], albedo=med["albedo"][0], emis=med["emis"][0], inflow=med["inflow"][:4])
    p2 = OL.make_problem(s2, med2)
    rng = np.random.default_rng(3)
    S0 = np.abs(rng.standard_normal(p3.shape))
    G = rng.standard_normal(p3.shape)
    r3 = O3.adjoint(S0, p3, 4, G)
    r2 = OA.adjoint(S0[:, :, 0], p2, 4, G[:, :, 0])
    for k in ("g_tau", "g_albedo", "g_emis"):
        assert np.abs(r3[k][0] - r2[k]).max() < 1e-12 * max(np.abs(r2[k]).max(), 1.0)
    assert np.abs(r3["lambda0"][:, :, 0] - r2["lambda0"]).max() < 1e-12 * np.abs(r2["lambda0"]).max()
