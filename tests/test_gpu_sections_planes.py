"""Parity of the HIP path with the FP64 oracle for the weights re-adapted every N
inline sections (Sec. 2, last paragraph) and for per-plane directional stencils
with graded line templates (Sec. 2 step 4, Fig. 4): forward outputs element by
element, stagewise fusion on the GPU's own S_m, and the adjoint."""
import numpy as np
import pytest

import gradcheck
from oracle import oracle as orc
from paper_2201_06174_amd import synth

pytestmark = pytest.mark.gpu

TOL_FP32 = 1e-5
TOL_GRAD = 1e-5


def _rel(x, ref):
    x, ref = np.asarray(x, np.float64), np.asarray(ref, np.float64)
    return float(np.max(np.abs(x - ref)) / max(np.max(np.abs(ref)), 1e-30))


@pytest.fixture(scope="module")
def torch_sal():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2201_06174_amd as sal
    return torch, sal


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _templates(s, kind):
    """Per-plane line templates: t plane along t, x plane along the crossline, y plane along
    the t-x diagonal (Fig. 4's three orientations), or along the inline."""
    if kind == "t_x_tx":
        dirs = ([s, 0, 0], [0, 0, s], [s, 0, s])
    else:
        dirs = ([s, 0, 0], [0, 0, s], [0, s, 0])
    return [orc.line_template(d, 2, 1.0) for d in dirs]


# shape, n, s, sections, fusion, masked, per-plane templates (or None: shared stencil)
CASES = [
    ((26, 35, 22), 8, 1, 4, "adapt_ls", True, None),
    ((30, 41, 27), 8, 2, 5, "adapt_ls", False, "t_x_tx"),
    ((36, 31, 29), 12, 2, 1, "adapt_ls", True, None),          # one weight group per inline section
    ((22, 40, 26), 16, 2, 7, "fixed", False, "t_x_il"),
    ((21, 19, 26), 8, 3, 100, "adapt_ls", True, None),        # N beyond the grid: one group
    ((24, 23, 20), 8, 1, 0, "equal", False, "t_x_tx"),        # per-plane templates alone
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_forward_matches_oracle(torch_sal, case):
    torch, sal = torch_sal
    shape, n, s, N, fusion, masked, tmpl = CASES[case]
    print("sections/planes forward case %d: shape %s n=%d s=%d N=%d %s" % (case, shape, n, s, N, tmpl), flush=True)
    rng = np.random.default_rng(100 + case)
    V = synth.make_volume(synth.VolumeSpec(shape, faults=[synth.centre_fault(shape)]), seed=200 + case)
    gs = orc.grid_shape(shape, s)
    D = (rng.uniform(size=gs) < 0.3).astype(np.float32)
    mask = (rng.uniform(size=gs) < 0.7).astype(np.uint8) if masked else None
    off = synth.cube_stencil(2 * s) if tmpl is None else synth.axis_stencil(s)
    planes = None if tmpl is None else _templates(s, tmpl)
    cfg = sal.Config(n=n, s=s, offsets=off, fusion=fusion, delta=1e-6, wfix=(0.2, 0.5, 0.3), sections=N,
                     planes=None if planes is None else [(o, w.astype(np.float32)) for o, w in planes])
    r = sal.saliency(_dev(torch, V), cfg, _dev(torch, D), None if mask is None else _dev(torch, mask))
    torch.cuda.synchronize()
    E, Sm, S, W = (r[k].cpu().numpy() for k in ("E", "Sm", "S", "W"))
    p = orc.Params(n=n, s=s, offsets=off, fusion=fusion, delta=1e-6, wfix=np.array([0.2, 0.5, 0.3]), D=D,
                   mask=mask, sections=N, planes=planes)
    o = orc.forward(V, p)
    for m in range(3):
        assert _rel(E[m], o["E"][m]) < TOL_FP32
        assert _rel(Sm[m], o["Sm"][m]) < TOL_FP32, m
    # stagewise: the oracle's fusion on the GPU's own S_m (its weights are then exact up
    # to the fixed-order FP64 sums), and the combine of those weights
    Wk = W.reshape(-1, 4)
    if N:
        Wo, fbo, _ = orc.fusion_weights_sections(Sm, N, D, mask, fusion, p.wfix, p.delta)
        assert Wk.shape[0] == orc.fuse_groups(gs[1], N)
        assert np.array_equal(Wk[:, 3] != 0, fbo != 0)
        So = orc.combine_sections(Sm, Wk[:, :3], N, shape, s)
    else:
        Wo, fbo, _ = orc.fusion_weights(Sm, D, mask, fusion, p.wfix, p.delta)
        Wo = Wo[None]
        So = orc.combine(Sm, Wk[0, :3], shape, s)
    assert np.max(np.abs(Wk[:, :3] - Wo)) < 1e-9 * max(np.abs(Wo).max(), 1e-30)
    assert _rel(S, So) < 1e-6
    # and end to end against the oracle's own maps
    assert np.max(np.abs(Wk[:, :3] - np.asarray(o["W"]).reshape(-1, 3))) < 1e-5 * np.abs(o["W"]).max()
    assert _rel(S, o["S"]) < TOL_FP32


def test_sections_at_or_beyond_the_grid_equal_one_fit(torch_sal):
    """N covering every inline section gives the plain fit bit for bit."""
    torch, sal = torch_sal
    shape = (30, 41, 27)
    V = synth.make_volume(synth.VolumeSpec(shape, faults=[synth.centre_fault(shape)]), seed=301)
    gs = orc.grid_shape(shape, 2)
    D = (np.random.default_rng(3).uniform(size=gs) < 0.3).astype(np.float32)
    Vd, Dd = _dev(torch, V), _dev(torch, D)
    base = sal.saliency(Vd, sal.Config(n=8, s=2, offsets=synth.cube_stencil(4), fusion="adapt_ls", delta=1e-6), Dd)
    for N in (gs[1], gs[1] + 3):
        r = sal.saliency(Vd, sal.Config(n=8, s=2, offsets=synth.cube_stencil(4), fusion="adapt_ls", delta=1e-6,
                                        sections=N), Dd)
        assert r["W"].shape == (1, 4)
        assert torch.equal(r["W"][0], base["W"]) and torch.equal(r["S"], base["S"])


BWD_CASES = [
    # shape, n, s, sections, fusion, masked, templates
    ((19, 21, 15), 8, 1, 3, "adapt_ls", True, None),
    ((22, 26, 18), 8, 2, 2, "equal", False, "t_x_tx"),
    ((20, 18, 17), 16, 1, 5, "adapt_ls", False, "t_x_il"),
    ((26, 22, 19), 12, 2, 0, "adapt_ls", True, "t_x_tx"),
]


@pytest.mark.parametrize("case", range(len(BWD_CASES)))
def test_backward_matches_oracle(torch_sal, case):
    torch, sal = torch_sal
    shape, n, s, N, fusion, masked, tmpl = BWD_CASES[case]
    print("sections/planes backward case %d: shape %s n=%d s=%d N=%d %s" % (case, shape, n, s, N, tmpl), flush=True)
    rng = np.random.default_rng(400 + case)
    V = synth.make_volume(synth.VolumeSpec(shape, faults=[synth.centre_fault(shape)]), seed=500 + case)
    gS = synth.loss_weights(shape, 600 + case)
    gs = orc.grid_shape(shape, s)
    D = (rng.uniform(size=gs) < 0.3).astype(np.float32)
    mask = (rng.uniform(size=gs) < 0.7).astype(np.uint8) if masked else None
    off = synth.axis_stencil(4 * s) if tmpl is None else synth.axis_stencil(s)
    planes = None if tmpl is None else _templates(s, tmpl)
    cfg = sal.Config(n=n, s=s, offsets=off, fusion=fusion, delta=1e-4, sections=N,
                     planes=None if planes is None else [(o, w.astype(np.float32)) for o, w in planes])
    Vd, Dd = _dev(torch, V), _dev(torch, D)
    Md = None if mask is None else _dev(torch, mask)
    r = sal.saliency(Vd, cfg, Dd, Md)
    gV = sal.backward(Vd, cfg, r["E"], r["Sm"], r["W"], _dev(torch, gS), Dd, Md).cpu().numpy()
    p = orc.Params(n=n, s=s, offsets=off, fusion=fusion, delta=1e-4, D=D, mask=mask, sections=N, planes=planes)
    ref, W, fb = orc.backward(V, p, gS)
    assert not np.any(fb)
    E = orc.features(V, n, s, "hann")
    amb = gradcheck.near_tie_voxels(E, shape, n, s, gradcheck.plane_stencils(off, None, planes), False, 1e-5)
    gradcheck.check_gradient(gV, ref, amb, TOL_GRAD)
