"""Maximum-size case: a volume whose grid planes (3 x 720 x 1024 x 1024 floats) and adjoint
tile workspace exceed 2^31 elements, so every kernel of the forward and the adjoint runs
its 64-bit index form.  Checks that hold at any size:

* locality: each output at distance >= 16 from the borders of a 64^3 crop depends only on
  samples inside the crop (window half-width 4, stencil reach 4 twice through the center-
  surround adjoint, half-width 4 again for the adjoint synthesis), so the large run and a run
  on the crop alone (32-bit index forms, tiles aligned the same way) agree there;
* oracle samples: E at a few interior centres against the FP64 oracle on the crop;
* the split-BF16 and FP16 feature kernels, large volume against crop.

Equal fusion keeps W independent of the volume.  The inputs are drawn on the device from a
seeded generator; about 100 GB of device memory is used."""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_2201_06174_amd import synth

pytestmark = pytest.mark.gpu

SHAPE = (720, 1024, 1024)
CROP0 = (640, 948, 952)   # multiples of the tile extents (8, 4, 4), near the far corner
C = 64                    # crop side
M = 16                    # compared interior starts this far inside the crop


@pytest.fixture(scope="module")
def torch_sal():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2201_06174_amd as sal
    return torch, sal


def _rel(x, ref):
    return float((x - ref).abs().max() / ref.abs().max().clamp_min(1e-30))


def test_int64_paths_match_crop_and_oracle(torch_sal):
    torch, sal = torch_sal
    print("large volume %s, crop at %s" % (SHAPE, CROP0), flush=True)
    assert 3 * int(np.prod(SHAPE)) >= 1 << 31
    gen = torch.Generator(device="cuda").manual_seed(7)
    V = torch.randn(SHAPE, generator=gen, device="cuda", dtype=torch.float32)
    gS = torch.rand(SHAPE, generator=gen, device="cuda", dtype=torch.float32)
    cfg = sal.Config(n=8, s=1, offsets=synth.axis_stencil(4), fusion="equal")
    r = sal.saliency(V, cfg)
    gV = sal.backward(V, cfg, r["E"], r["Sm"], r["W"], gS)
    torch.cuda.synchronize()

    t0, i0, x0 = CROP0
    box = (slice(t0, t0 + C), slice(i0, i0 + C), slice(x0, x0 + C))
    inner = (slice(t0 + M, t0 + C - M), slice(i0 + M, i0 + C - M), slice(x0 + M, x0 + C - M))
    Vc = V[box].contiguous()
    rc = sal.saliency(Vc, cfg)
    gVc = sal.backward(Vc, cfg, rc["E"], rc["Sm"], rc["W"], gS[box].contiguous())
    torch.cuda.synchronize()
    ci = (slice(M, C - M),) * 3

    errs = {
        "E": _rel(r["E"][(slice(None),) + inner], rc["E"][(slice(None),) + ci]),
        "Sm": _rel(r["Sm"][(slice(None),) + inner], rc["Sm"][(slice(None),) + ci]),
        "S": _rel(r["S"][inner], rc["S"][ci]),
        "gV": _rel(gV[inner], gVc[ci]),
    }
    print("  large vs crop, interior rel diff: %s" % ", ".join("%s %.2e" % kv for kv in errs.items()), flush=True)
    assert errs["E"] <= 1e-6 and errs["Sm"] <= 1e-6 and errs["S"] <= 1e-6
    assert errs["gV"] <= 1e-5

    # E at interior centres against the FP64 oracle (windows inside the crop: no reflection)
    rng = np.random.default_rng(11)
    g_rel = rng.integers(M, C - M, size=(8, 3))
    ref = orc.features_at(Vc.cpu().numpy(), 8, 1, "hann", g_rel)
    got = np.stack([r["E"][:, t0 + a, i0 + b, x0 + c].cpu().numpy() for a, b, c in g_rel])
    err = float(np.abs(got - ref).max() / np.abs(ref).max())
    print("  E vs oracle at 8 centres: %.2e" % err, flush=True)
    assert err <= 1e-5

    # the reduced-precision feature kernels take the same 64-bit paths
    del gV, gVc
    for prec in ("split_bf16", "fp16"):
        El = sal.project(V, 8, 1, "hann", prec)
        Ec = sal.project(Vc, 8, 1, "hann", prec)
        e = _rel(El[(slice(None),) + inner], Ec[(slice(None),) + ci])
        print("  %s features, large vs crop: %.2e" % (prec, e), flush=True)
        assert e <= 1e-6
        del El, Ec

    del V, gS, r, rc
    torch.cuda.empty_cache()
