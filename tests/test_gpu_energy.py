"""The energy feature (mean of |F_m|^2, the spectral energy of each projection) on the
GPU against the FP64 oracle: features element by element at every window side, the whole
forward with adapted fusion, and the adjoint (Y = 2 c(k) F(k))."""
import numpy as np
import pytest

import gradcheck
from oracle import oracle as orc
from paper_2201_06174_amd import synth

pytestmark = pytest.mark.gpu

TOL_FP32 = 1e-5


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


CASES = [((37, 29, 23), 8, 1, "hann"), ((30, 41, 27), 8, 2, "hann"), ((45, 26, 35), 16, 2, "hann"),
         ((17, 23, 19), 16, 1, "rect"), ((36, 31, 29), 12, 2, "hann"), ((40, 9, 13), 4, 1, "hann"),
         ((33, 38, 29), 12, 4, "hann"), ((8, 8, 8), 16, 7, "hann")]


@pytest.mark.parametrize("shape,n,s,window", CASES)
def test_energy_features(torch_sal, shape, n, s, window):
    torch, sal = torch_sal
    print("energy features shape=%s n=%d s=%d %s" % (shape, n, s, window), flush=True)
    V = np.random.default_rng(sum(shape) + 3 * n).standard_normal(shape).astype(np.float32)
    E = sal.project(_dev(torch, V), n, s, window, "fp32", "energy").cpu().numpy()
    ref = orc.features(V, n, s, window, feature="energy")
    for m in range(3):
        assert _rel(E[m], ref[m]) < TOL_FP32, m


def test_energy_forward_and_adjoint(torch_sal):
    torch, sal = torch_sal
    shape, n, s = (26, 23, 21), 8, 1
    V, M = synth.make_volume(synth.VolumeSpec(shape, faults=[synth.centre_fault(shape)]), 41, with_mask=True)
    D, mask = synth.desired_map(M, s)
    gS = synth.loss_weights(shape, 42)
    off = synth.axis_stencil(4)
    cfg = sal.Config(n=n, s=s, offsets=off, fusion="adapt_ls", delta=1e-6, feature="energy")
    Vd, Dd, Md = _dev(torch, V), _dev(torch, D), _dev(torch, mask)
    r = sal.saliency(Vd, cfg, Dd, Md)
    p = orc.Params(n=n, s=s, offsets=off, fusion="adapt_ls", delta=1e-6, D=D, mask=mask, feature="energy")
    o = orc.forward(V, p)
    assert _rel(r["E"].cpu().numpy(), o["E"]) < TOL_FP32
    assert _rel(r["Sm"].cpu().numpy(), o["Sm"]) < TOL_FP32
    W = r["W"].cpu().numpy()
    assert W[3] == 0 and _rel(W[:3], o["W"]) < TOL_FP32
    assert _rel(r["S"].cpu().numpy(), o["S"]) < TOL_FP32
    gV = sal.backward(Vd, cfg, r["E"], r["Sm"], r["W"], _dev(torch, gS), Dd, Md).cpu().numpy()
    ref, _, fb = orc.backward(V, p, gS)
    assert fb == 0
    amb = gradcheck.near_tie_voxels(o["E"], shape, n, s, gradcheck.plane_stencils(off, None, None), False,
                                    4e-6 * np.abs(o["E"]).max())
    gradcheck.check_gradient(gV, ref, amb, TOL_FP32)


@pytest.mark.parametrize("n,s", [(16, 2), (12, 3), (4, 1)])
def test_energy_adjoint_other_sides(torch_sal, n, s):
    torch, sal = torch_sal
    shape = (30, 27, 25)
    print("energy adjoint n=%d s=%d" % (n, s), flush=True)
    rng = np.random.default_rng(n * 10 + s)
    V = rng.standard_normal(shape).astype(np.float32)
    gS = rng.uniform(size=shape).astype(np.float32)
    off = synth.cube_stencil(2 * s)
    cfg = sal.Config(n=n, s=s, offsets=off, fusion="equal", feature="energy")
    Vd = _dev(torch, V)
    r = sal.saliency(Vd, cfg)
    gV = sal.backward(Vd, cfg, r["E"], r["Sm"], r["W"], _dev(torch, gS)).cpu().numpy()
    p = orc.Params(n=n, s=s, offsets=off, feature="energy")
    ref, _, _ = orc.backward(V, p, gS)
    E = orc.features(V, n, s, "hann", feature="energy")
    amb = gradcheck.near_tie_voxels(E, shape, n, s, gradcheck.plane_stencils(off, None, None), False,
                                    4e-6 * np.abs(E).max())
    gradcheck.check_gradient(gV, ref, amb, TOL_FP32)
