"""Batched form: many uneven subvolumes with mixed window sides in one
captured graph of persistent kernels.  Every member's outputs must equal the
single-volume calls bit for bit (same per-window arithmetic), graph replays
must be idempotent, and sampled members are checked against the oracle."""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_2201_06174_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_sal():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2201_06174_amd as sal
    return torch, sal


def _members(torch, sal, count, precision="fp32", fusion="adapt_ls"):
    out = []
    for i in range(count):
        w = synth.workload("batch", i)
        V, M = synth.make_volume(w.spec, w.seed, with_mask=True)
        D, mask = synth.desired_map(M, w.s)
        cfg = sal.Config(n=w.n, s=w.s, offsets=w.offsets, fusion=fusion if i % 3 else "equal", delta=1e-6,
                         precision=precision)
        out.append({"V": torch.from_numpy(V).cuda(), "cfg": cfg, "D": torch.from_numpy(D).cuda(),
                    "mask": torch.from_numpy(mask).cuda(), "host": V})
    return out


def _same_as_single(torch, sal, plan, members):
    for i, m in enumerate(members):
        r = sal.saliency(m["V"], m["cfg"], m["D"], m["mask"])
        o = plan.output(i)
        for k in ("E", "Sm", "S", "W"):
            assert torch.equal(o[k], r[k]), (i, k)


def test_plan_matches_single_calls(torch_sal):
    torch, sal = torch_sal
    members = _members(torch, sal, 24)
    plan = sal.Plan(members)
    print(plan.describe())
    plan.launch()
    torch.cuda.synchronize()
    _same_as_single(torch, sal, plan, members)
    # replay: identical results
    first = [{k: v.clone() for k, v in plan.output(i).items()} for i in range(len(members))]
    for _ in range(2):
        plan.launch()
        torch.cuda.synchronize()
        for i in range(len(members)):
            for k in ("E", "Sm", "S", "W"):
                assert torch.equal(plan.output(i)[k], first[i][k])
    plan.close()


def test_plan_autotune_and_direct_launch(torch_sal):
    torch, sal = torch_sal
    members = _members(torch, sal, 12)
    tuned = sal.Plan(members, autotune=True)
    print(tuned.describe())
    tuned.launch()
    direct = sal.Plan(members, graph=False)
    direct.launch()
    torch.cuda.synchronize()
    for i in range(len(members)):
        for k in ("E", "Sm", "S", "W"):
            assert torch.equal(tuned.output(i)[k], direct.output(i)[k]), (i, k)
    _same_as_single(torch, sal, direct, members)
    tuned.close()
    direct.close()


def test_plan_autotune_reduced_precision(torch_sal):
    """Autotuning times every candidate tile depth, so the reduced-precision kernels also
    run with tiles shallower than the full depth; the tuned plan still equals the single calls."""
    torch, sal = torch_sal
    members = _members(torch, sal, 6, precision="split_bf16")
    plan = sal.Plan(members, autotune=True)
    print(plan.describe())
    plan.launch()
    torch.cuda.synchronize()
    _same_as_single(torch, sal, plan, members)
    plan.close()


@pytest.mark.parametrize("precision", ["split_bf16", "fp16"])
def test_plan_reduced_precision(torch_sal, precision):
    torch, sal = torch_sal
    members = _members(torch, sal, 9, precision=precision)
    plan = sal.Plan(members)
    plan.launch()
    torch.cuda.synchronize()
    _same_as_single(torch, sal, plan, members)
    plan.close()


def test_full_batch_and_oracle_samples(torch_sal):
    """All 96 members (axes uniform in 32..160, n in {8, 12, 16}) in one plan;
    four members checked at sampled grid points against the oracle."""
    torch, sal = torch_sal
    members = _members(torch, sal, 96)
    plan = sal.Plan(members)
    plan.launch()
    torch.cuda.synchronize()
    rng = np.random.default_rng(96)
    for i in (0, 17, 50, 95):
        m = members[i]
        w = synth.workload("batch", i)
        o = plan.output(i)
        gs = o["E"].shape[1:]
        g = np.stack([rng.integers(0, N, 24) for N in gs], 1).astype(np.int64)
        Sr, Er = orc.saliency_at(m["host"], w.n, w.s, "hann", w.offsets, None, False, g)
        E = o["E"][:, g[:, 0], g[:, 1], g[:, 2]].T.cpu().numpy()
        S = o["Sm"][:, g[:, 0], g[:, 1], g[:, 2]].T.cpu().numpy()
        assert np.max(np.abs(E - Er)) / np.max(np.abs(Er)) < 1e-5
        assert np.max(np.abs(S - Sr)) / np.max(np.abs(Sr)) < 1e-5
    _same_as_single(torch, sal, plan, members[:6])
    plan.close()


def test_plan_status_word(torch_sal):
    """sal_plan_status: the number of members whose adapted fit fell back to equal weights
    and the lowest of them, from the device status word the plan's graph writes."""
    torch, sal = torch_sal
    members = []
    for i, fallback in enumerate((False, True, False, True)):
        shape = (20 + i, 18, 22)
        V = synth.make_volume(synth.VolumeSpec(shape, faults=[synth.centre_fault(shape)]), seed=900 + i)
        gs = sal.grid_shape(shape, 1)
        D = np.ones(gs, np.float32)
        # a member whose fit mask is empty has no Gram matrix to solve: equal weights, flagged
        mask = np.zeros(gs, np.uint8) if fallback else np.ones(gs, np.uint8)
        cfg = sal.Config(n=8, s=1, offsets=synth.axis_stencil(4), fusion="adapt_ls", delta=0.0)
        members.append({"V": torch.from_numpy(V).cuda(), "cfg": cfg, "D": torch.from_numpy(D).cuda(),
                        "mask": torch.from_numpy(mask).cuda()})
    plan = sal.Plan(members)
    plan.launch()
    assert plan.status() == (2, 1)
    for i in range(4):
        assert plan.output(i)["W"][3].item() == (1.0 if i in (1, 3) else 0.0)
    plan.close()


def test_autotune_cache_persists_across_processes(tmp_path):
    """SAL_AUTOTUNE_CACHE: a first process times the candidate tile depths and appends them
    to the file; a second process on the same architecture reads them instead of timing."""
    import os
    import subprocess
    import sys
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    script = (
        "import sys; sys.path.insert(0, %r)\n"
        "import torch\n"
        "import paper_2201_06174_amd as sal\n"
        "from paper_2201_06174_amd import synth\n"
        "ms = []\n"
        "for i, shape in enumerate(((40, 36, 44), (44, 40, 36))):\n"
        "    V = synth.make_volume(synth.VolumeSpec(shape, faults=[synth.centre_fault(shape)]), 300 + i)\n"
        "    ms.append({'V': torch.from_numpy(V).cuda(), 'cfg': sal.Config(n=16, s=2, offsets=synth.axis_stencil(8))})\n"
        "p = sal.Plan(ms, autotune=True)\n"
        "print(p.describe())\n" % root)
    env = dict(os.environ, SAL_AUTOTUNE_CACHE=str(tmp_path / "tune.txt"))
    first = subprocess.run([sys.executable, "-c", script], env=env, capture_output=True, text=True, timeout=110)
    print(first.stdout, first.stderr[-2000:])
    assert first.returncode == 0 and "CT=" in first.stdout
    lines = (tmp_path / "tune.txt").read_text().split("\n")
    assert lines[0].startswith("gfx") and len(lines[0].split()) == 7
    second = subprocess.run([sys.executable, "-c", script], env=env, capture_output=True, text=True, timeout=110)
    print(second.stdout)
    assert second.returncode == 0 and "cached in" in second.stdout and "CT=" not in second.stdout
