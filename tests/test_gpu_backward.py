"""Parity of the hand-written HIP adjoint with the FP64 oracle gradient, and
central finite differences through the HIP forward.

sgn(E(g) - E(g+o)) decides which way each center-surround term pulls; where the
oracle's own difference is within a hair of zero the two sides may take
different (equally valid) subgradients.  Such near-tie windows are found from
the oracle's features and the voxels they reach are left out of the
element-wise comparison (the test requires them to be rare)."""
import numpy as np
import pytest

import gradcheck
from oracle import oracle as orc
from paper_2201_06174_amd import synth

pytestmark = pytest.mark.gpu

TOL_GRAD = 1e-5


@pytest.fixture(scope="module")
def torch_sal():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2201_06174_amd as sal
    return torch, sal


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


CASES = [
    # shape, n, s, offsets, fusion, literal, window
    ((19, 17, 15), 8, 1, synth.axis_stencil(4), "equal", False, "hann"),
    ((22, 18, 26), 8, 2, synth.cube_stencil(2), "adapt_ls", False, "hann"),
    ((17, 21, 20), 8, 3, synth.axis_stencil(3), "fixed", True, "rect"),
    ((30, 27, 25), 16, 2, synth.cube_stencil(8), "equal", False, "hann"),
    ((20, 18, 17), 16, 1, synth.axis_stencil(8), "adapt_ls", False, "hann"),
    ((26, 22, 19), 12, 2, synth.axis_stencil(6), "equal", False, "hann"),
    ((25, 24, 23), 12, 3, synth.axis_stencil(6), "fixed", False, "hann"),
    ((23, 19, 21), 12, 1, synth.cube_stencil(3), "adapt_ls", False, "hann"),
    ((13, 10, 9), 4, 1, synth.axis_stencil(2), "equal", False, "hann"),
    ((8, 9, 8), 16, 2, synth.axis_stencil(2), "equal", False, "hann"),   # axes of n/2 voxels
    # wide strides: shallower adjoint tiles (4, 2 or 1 t-centres) that fit the LDS
    ((37, 33, 35), 12, 4, synth.axis_stencil(8), "equal", False, "hann"),
    ((33, 36, 31), 12, 5, synth.cube_stencil(5), "adapt_ls", False, "hann"),
    ((34, 31, 36), 16, 3, synth.axis_stencil(6), "equal", False, "hann"),
    ((39, 34, 37), 16, 4, synth.cube_stencil(8), "fixed", False, "hann"),
    ((41, 38, 36), 16, 5, synth.axis_stencil(10), "equal", True, "rect"),
    ((40, 37, 43), 16, 6, synth.axis_stencil(6), "equal", False, "hann"),
    ((45, 39, 41), 16, 7, synth.axis_stencil(7), "adapt_ls", False, "hann"),
    # one-sided stencils (no offset pairs with its negation), both forms of Eq. 3
    ((18, 16, 17), 8, 1, np.array([[1, 0, 0], [0, 2, 0], [0, 0, -1], [1, 1, 1], [-2, 0, 1]]), "equal", False, "hann"),
    ((16, 19, 18), 8, 2, np.array([[2, 0, 0], [0, -2, 2], [0, 0, 4], [-4, 2, 0]]), "adapt_ls", True, "hann"),
]


@pytest.mark.parametrize("shape,n,s,off,fusion,literal,window", CASES)
def test_backward_matches_oracle(torch_sal, shape, n, s, off, fusion, literal, window):
    torch, sal = torch_sal
    print("backward shape=%s n=%d s=%d fusion=%s" % (shape, n, s, fusion), flush=True)
    rng = np.random.default_rng(sum(shape) * 7 + n)
    V = rng.standard_normal(shape).astype(np.float32)
    gS = rng.uniform(size=shape).astype(np.float32)
    gs = orc.grid_shape(shape, s)
    D = (rng.uniform(size=gs) < 0.3).astype(np.float32)
    mask = (rng.uniform(size=gs) < 0.7).astype(np.uint8)
    wfix = (0.5, 0.3, 0.2)
    cfg = sal.Config(n=n, s=s, window=window, offsets=off, literal=literal, fusion=fusion, wfix=wfix, delta=1e-4)
    Vd, Dd, Md = _dev(torch, V), _dev(torch, D), _dev(torch, mask)
    r = sal.saliency(Vd, cfg, Dd, Md)
    gV = sal.backward(Vd, cfg, r["E"], r["Sm"], r["W"], _dev(torch, gS), Dd, Md).cpu().numpy()
    p = orc.Params(n=n, s=s, window=window, offsets=off, literal=literal, fusion=fusion, wfix=np.array(wfix),
                   delta=1e-4, D=D, mask=mask)
    ref, W, fb = orc.backward(V, p, gS)
    assert fb == 0
    E = orc.features(V, n, s, window)
    amb = gradcheck.near_tie_voxels(E, shape, n, s, gradcheck.plane_stencils(off, None, None), literal,
                                    4e-6 * np.abs(E).max())
    gradcheck.check_gradient(gV, ref, amb, TOL_GRAD)


def test_isolated_points(torch_sal):
    """Degenerate stencil: every neighbour lies outside the 8^3 grid, so Q = 0 at every point,
    S_m = 0 (Eq. 3 with no terms) and no gradient reaches V."""
    torch, sal = torch_sal
    print("isolated points (8, 8, 8) offset 8", flush=True)
    shape, off = (8, 8, 8), synth.axis_stencil(8)
    rng = np.random.default_rng(3)
    V = rng.standard_normal(shape).astype(np.float32)
    gS = rng.uniform(size=shape).astype(np.float32)
    cfg = sal.Config(n=8, s=1, offsets=off, fusion="equal")
    r = sal.saliency(_dev(torch, V), cfg)
    gV = sal.backward(_dev(torch, V), cfg, r["E"], r["Sm"], r["W"], _dev(torch, gS)).cpu().numpy()
    p = orc.Params(n=8, s=1, offsets=off, fusion="equal")
    ref, W, fb = orc.backward(V, p, gS)
    assert not np.any(ref)
    assert not r["Sm"].cpu().numpy().any() and not r["S"].cpu().numpy().any()
    assert not np.any(gV)
    assert r["E"].abs().max().item() > 0


def test_autograd_function(torch_sal):
    torch, sal = torch_sal
    shape = (20, 16, 18)
    rng = np.random.default_rng(3)
    V = _dev(torch, rng.standard_normal(shape).astype(np.float32)).requires_grad_(True)
    wgt = _dev(torch, rng.uniform(size=shape).astype(np.float32))
    cfg = sal.Config(n=8, s=1, offsets=synth.axis_stencil(4))
    S = sal.SaliencyFn.apply(V, cfg)
    (S * wgt).sum().backward()
    with torch.no_grad():
        r = sal.saliency(V.detach(), cfg)
        gV = sal.backward(V.detach(), cfg, r["E"], r["Sm"], r["W"], wgt)
    assert torch.equal(V.grad, gV)


def test_backward_deterministic(torch_sal):
    torch, sal = torch_sal
    w = synth.workload("small")
    V = synth.make_volume(w.spec, w.seed)
    Vd = _dev(torch, V)
    gS = _dev(torch, synth.loss_weights(V.shape))
    cfg = sal.Config(n=w.n, s=w.s, offsets=w.offsets)
    r = sal.saliency(Vd, cfg)
    a = sal.backward(Vd, cfg, r["E"], r["Sm"], r["W"], gS)
    b = sal.backward(Vd, cfg, r["E"], r["Sm"], r["W"], gS)
    assert torch.equal(a, b)


def test_grad_workload_oracle_and_fd(torch_sal):
    """128^3 faulted volume, window 8^3, loss sum(S * U(0,1) weights): the
    adjoint against the FP64 oracle gradient at 64 random voxels, and against
    central differences (h = 1e-3) of the HIP forward at the same 64 voxels."""
    torch, sal = torch_sal
    w = synth.workload("grad")
    V = synth.make_volume(w.spec, w.seed)
    gS = synth.loss_weights(V.shape, 5001)
    cfg = sal.Config(n=w.n, s=w.s, offsets=w.offsets, fusion="equal")
    Vd, gSd = _dev(torch, V), _dev(torch, gS)
    r = sal.saliency(Vd, cfg)
    gV = sal.backward(Vd, cfg, r["E"], r["Sm"], r["W"], gSd).cpu().numpy()
    rng = np.random.default_rng(64)
    pts = np.stack([rng.integers(0, N, 64) for N in V.shape], 1).astype(np.int64)
    pts[:4] = [[0, 0, 0], [127, 127, 127], [0, 64, 127], [3, 125, 2]]
    p = orc.Params(n=w.n, s=w.s, offsets=w.offsets)
    ref = orc.backward_at(V, p, gS, pts)
    got = gV[tuple(pts.T)]
    scale = np.max(np.abs(ref))
    rel = np.abs(got - ref) / scale
    over = np.flatnonzero(rel > TOL_GRAD)
    print("oracle: max rel err over 64 voxels %.3e, %d above %.0e" % (rel.max(), len(over), TOL_GRAD), flush=True)
    # a voxel over the tolerance must sit where a center-surround difference is at a tie
    # (the two sides may then take different subgradients), found from oracle features
    E_scale = float(r["E"].abs().max().item())
    for k in over:
        assert gradcheck.voxel_explained_by_tie(V, w.n, w.s, "hann", w.offsets, None, False, pts[k],
                                                4e-6 * E_scale), (pts[k], rel[k])
    assert len(over) <= 2, rel
    # central differences through the HIP forward
    h = 1e-3
    gS64 = gS.astype(np.float64)
    fd_err = []
    skipped = 0
    for q in pts:
        vals = []
        for d in (-h, 0.0, h):
            Vp = V.copy()
            Vp[tuple(q)] += np.float32(d)
            S = sal.saliency(_dev(torch, Vp), cfg)["S"].cpu().numpy().astype(np.float64)
            vals.append(float(np.sum(S * gS64)))
        bwd, fwd = (vals[1] - vals[0]) / h, (vals[2] - vals[1]) / h
        if abs(fwd - bwd) > 0.2 * (abs(fwd) + abs(bwd)) + 1e-3:
            skipped += 1
            continue
        fd = (vals[2] - vals[0]) / (2 * h)
        fd_err.append(abs(fd - gV[tuple(q)]) / (abs(gV[tuple(q)]) + 1e-2 * scale))
    print("finite differences: %d checked, %d skipped (kinks), median rel err %.3e, max %.3e" % (
        len(fd_err), skipped, float(np.median(fd_err)), max(fd_err)))
    # h = 1e-3 is about 1/60 of the data's standard deviation, so the central difference
    # itself carries a curvature error of a few percent (the oracle-side pin shows the same
    # at this step); the 1e-5 gate is the comparison with the oracle gradient above.
    assert len(fd_err) >= 48 and float(np.median(fd_err)) < 1e-2 and max(fd_err) < 0.15
