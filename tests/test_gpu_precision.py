"""Reduced-precision DFT contractions against the FP64 oracle, per output.

SPLIT_BF16 (hi + lo bfloat16 operands, three products, fp32 accumulate) is gated
at 1e-3 relative per output (E, S_m, W, S); FP16 (one product) is stated, with a
loose sanity bound only.  Relative error = max|x - ref| / max|ref| per output.
Small volumes are compared element by element through the whole forward with
adapted fusion; the 512^3 salt-dome volume on the middle inline section (where the
weights are fitted, so the oracle's W there is the oracle's W of the volume) and
at sampled grid points including corners and faces."""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_2201_06174_amd import synth

pytestmark = pytest.mark.gpu

TOL = {"fp32": 1e-5, "split_bf16": 1e-3, "fp16": 2e-2}


@pytest.fixture(scope="module")
def torch_sal():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2201_06174_amd as sal
    return torch, sal


def _rel(x, ref):
    x, ref = np.asarray(x, np.float64), np.asarray(ref, np.float64)
    return float(np.max(np.abs(x - ref)) / max(np.max(np.abs(ref)), 1e-30))


CASES = [((37, 29, 23), 8, 1, "hann"), ((30, 41, 27), 8, 2, "hann"), ((45, 26, 35), 16, 2, "hann"),
         ((17, 23, 19), 16, 1, "rect"), ((36, 31, 29), 12, 2, "hann"), ((21, 19, 26), 12, 3, "hann"),
         ((40, 9, 13), 4, 1, "hann"), ((8, 8, 8), 16, 7, "hann"),
         # split-bf16 at n = 16, s = 3 takes a shallower tile than the full depth (LDS), the
         # general kernel with a compile-time stride; fp16 keeps the full-depth one
         ((50, 23, 29), 16, 3, "hann"),
         # a run-time stride (no compile-time instance) over several tiles
         ((33, 38, 29), 12, 4, "hann"), ((41, 35, 44), 16, 5, "hann")]


@pytest.mark.parametrize("precision", ["split_bf16", "fp16"])
@pytest.mark.parametrize("shape,n,s,window", CASES)
def test_forward_reduced_precision(torch_sal, precision, shape, n, s, window):
    """The whole forward (adapted fusion on a desired map) in each precision against the
    oracle: E, S_m, W and S, element by element."""
    torch, sal = torch_sal
    print("forward %s shape=%s n=%d s=%d" % (precision, shape, n, s), flush=True)
    V, M = synth.make_volume(synth.VolumeSpec(shape, faults=[synth.centre_fault(shape)]), sum(shape) + n,
                             with_mask=True)
    gs = orc.grid_shape(shape, s)
    D = np.random.default_rng(n).uniform(size=gs).astype(np.float32)
    off = synth.axis_stencil(2 * s)
    cfg = sal.Config(n=n, s=s, window=window, precision=precision, offsets=off, fusion="adapt_ls", delta=1e-6)
    r = sal.saliency(torch.from_numpy(V).cuda(), cfg, torch.from_numpy(D).cuda())
    o = orc.forward(V, orc.Params(n=n, s=s, window=window, offsets=off, fusion="adapt_ls", delta=1e-6, D=D))
    W = r["W"].cpu().numpy()
    assert W[3] == 0 and o["fallback"] == 0
    errs = {"E": _rel(r["E"].cpu().numpy(), o["E"]), "Sm": _rel(r["Sm"].cpu().numpy(), o["Sm"]),
            "W": _rel(W[:3], o["W"]), "S": _rel(r["S"].cpu().numpy(), o["S"])}
    print("  rel err per output: %s" % ", ".join("%s %.2e" % kv for kv in errs.items()), flush=True)
    assert max(errs.values()) < TOL[precision]


@pytest.mark.timeout(400)
def test_salt_workload_per_output(torch_sal):
    """512^3 salt-dome volume, window 16^3, stride 2, 26 neighbours at offset 8, adapted
    weights fitted on the middle inline section: per precision, E and S_m on that section
    and at 192 sampled grid points (corners and faces among them), W against the oracle's
    fit, S at sampled voxels of that section, all against the FP64 oracle; the GPU's fusion
    step also stagewise (the oracle's fit and combine on the GPU's own S_m)."""
    torch, sal = torch_sal
    w = synth.workload("salt")
    V, M = synth.make_volume(w.spec, w.seed, with_mask=True)
    D, mask = synth.desired_map(M, w.s)
    gs = orc.grid_shape(V.shape, w.s)
    mid = gs[1] // 2
    assert mask.sum() == mask[:, mid, :].sum()  # the fit uses the middle section only
    print("oracle on the middle inline section of the salt volume", flush=True)
    E_o, S_o = orc.saliency_inline_plane(V, w.n, w.s, "hann", w.offsets, None, False, mid)
    W_o, fb_o, _ = orc.fusion_weights(S_o, D[:, mid, :], mask[:, mid, :], "adapt_ls", delta=1e-6)
    assert fb_o == 0
    rng = np.random.default_rng(11)
    g = np.stack([rng.integers(0, N, 192) for N in gs], 1).astype(np.int64)
    g[:8] = [[a, b, c] for a in (0, gs[0] - 1) for b in (0, gs[1] - 1) for c in (0, gs[2] - 1)]
    g[8:14] = [[0, mid, 7], [gs[0] - 1, 3, 9], [5, 0, 11], [9, gs[1] - 1, 2], [4, 6, 0], [100, 7, gs[2] - 1]]
    Sg_o, Eg_o = orc.saliency_at(V, w.n, w.s, "hann", w.offsets, None, False, g)
    # voxels whose nearest centre lies on the middle section
    v = np.stack([rng.integers(0, V.shape[0], 4096), np.full(4096, mid * w.s), rng.integers(0, V.shape[2], 4096)], 1)
    gv = np.minimum(v // w.s, np.array(gs) - 1)
    Vd, Dd, Md = (torch.from_numpy(a).cuda() for a in (V, D, mask))
    for prec in ("fp32", "split_bf16", "fp16"):
        cfg = sal.Config(n=w.n, s=w.s, precision=prec, offsets=w.offsets, fusion="adapt_ls", delta=1e-6)
        r = sal.saliency(Vd, cfg, Dd, Md)
        E, Sm, W = r["E"].cpu().numpy(), r["Sm"].cpu().numpy(), r["W"].cpu().numpy()
        Sv = r["S"][v[:, 0], v[:, 1], v[:, 2]].cpu().numpy()
        S_ref = (W_o[:, None] * S_o[:, gv[:, 0], gv[:, 2]]).sum(0)
        errs = {"E": max(_rel(E[:, :, mid, :], E_o), _rel(E[:, g[:, 0], g[:, 1], g[:, 2]].T, Eg_o)),
                "Sm": max(_rel(Sm[:, :, mid, :], S_o), _rel(Sm[:, g[:, 0], g[:, 1], g[:, 2]].T, Sg_o)),
                "W": _rel(W[:3], W_o), "S": _rel(Sv, S_ref)}
        print("salt %s: rel err per output: %s" % (prec, ", ".join("%s %.2e" % kv for kv in errs.items())),
              flush=True)
        assert W[3] == 0 and max(errs.values()) < TOL[prec]
        # stagewise fusion on the GPU's own maps
        Ws, fb, _ = orc.fusion_weights(Sm, D, mask, "adapt_ls", delta=1e-6)
        assert fb == 0 and np.max(np.abs(W[:3] - Ws)) < 1e-9 * np.abs(Ws).max()
        # the combine of the middle section alone: a volume w.s inline samples thick whose
        # single grid section is the middle one
        S_mid = orc.combine(Sm[:, :, mid:mid + 1, :], W[:3], (V.shape[0], w.s, V.shape[2]), w.s)
        assert _rel(Sv, S_mid[v[:, 0], 0, v[:, 2]]) < 1e-6
        del r, E, Sm
        torch.cuda.empty_cache()
