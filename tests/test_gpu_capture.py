"""Graph capture of the C-ABI calls.  In a fresh process (so the constant tables are
not uploaded yet): a first call inside a stream capture before sal_init returns
SAL_ERR_STATE and leaves the capture intact; after sal_init the whole forward
(sal_project -> sal_center_surround -> sal_fuse, adapted weights) and sal_backward
are captured in one graph with torch.cuda.graph, and every replay, with eager work
and synchronisations between replays, matches the direct calls bit for bit."""
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = r'''
import ctypes, sys
import numpy as np
import torch
sys.path.insert(0, sys.argv[1])
import paper_2201_06174_amd as sal
from paper_2201_06174_amd import _lib, synth

lib = _lib.load()
hip = ctypes.CDLL("libamdhip64.so")
torch.cuda.init()
shape = (40, 37, 33)
V, M = synth.make_volume(synth.VolumeSpec(shape, faults=[synth.centre_fault(shape)]), 11, with_mask=True)
D, mask = synth.desired_map(M, 2)
Vd = torch.from_numpy(V).cuda()
Dd, Md = torch.from_numpy(D).cuda(), torch.from_numpy(mask).cuda()
E = torch.empty((3,) + sal.grid_shape(shape, 2), dtype=torch.float32, device="cuda")
torch.cuda.synchronize()

# 1. a first call inside a capture, before sal_init: SAL_ERR_STATE, nothing enqueued
s = torch.cuda.Stream()
h = ctypes.c_void_p(s.cuda_stream)
assert hip.hipStreamBeginCapture(h, 1) == 0          # thread-local capture mode
spec = _lib.make_spec(16, 2)
rc = lib.sal_project(ctypes.c_void_p(Vd.data_ptr()), shape[0], shape[1], shape[2], spec, ctypes.c_void_p(E.data_ptr()), h)
graph = ctypes.c_void_p()
rc_end = hip.hipStreamEndCapture(h, ctypes.byref(graph))
print("first call in a capture before sal_init:", _lib.STATUS_NAMES[rc], lib.sal_last_error().decode(), flush=True)
assert _lib.STATUS_NAMES[rc] == "SAL_ERR_STATE", rc
assert rc_end == 0, rc_end
assert hip.hipGraphDestroy(graph) == 0

# 2. after init: forward and backward captured in one graph, no eager call before
sal.init()
gS = torch.from_numpy(synth.loss_weights(shape, 77)).cuda()
for n, s_, off in ((16, 2, synth.cube_stencil(4)), (8, 1, synth.axis_stencil(4))):
    cfg = sal.Config(n=n, s=s_, offsets=off, fusion="adapt_ls", delta=1e-6)
    Dn, Mn = synth.desired_map(M, s_)
    Dnd, Mnd = torch.from_numpy(Dn).cuda(), torch.from_numpy(Mn).cuda()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        r = sal.saliency(Vd, cfg, Dnd, Mnd)
        gV = sal.backward(Vd, cfg, r["E"], r["Sm"], r["W"], gS, Dnd, Mnd)
    ref = sal.saliency(Vd, cfg, Dnd, Mnd)
    gref = sal.backward(Vd, cfg, ref["E"], ref["Sm"], ref["W"], gS, Dnd, Mnd)
    torch.cuda.synchronize()
    junk = torch.zeros(1 << 20, device="cuda")
    for rep in range(3):
        for k in ("E", "Sm", "S", "W"):
            r[k].fill_(float("nan"))
        gV.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        junk.add_(1.0)                                # eager work between the replays
        torch.cuda.synchronize()
        for k in ("E", "Sm", "S", "W"):
            assert torch.equal(r[k], ref[k]), (n, rep, k)
        assert torch.equal(gV, gref), (n, rep)
    print("n=%d s=%d: 3 replays match the direct calls bit for bit" % (n, s_), flush=True)
print("CAPTURE_OK", flush=True)
'''


def test_capture_in_a_fresh_process():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    print("graph capture in a fresh process", flush=True)
    p = subprocess.run([sys.executable, "-c", SCRIPT, ROOT], stdout=subprocess.PIPE, stderr=subprocess.STDOUT,
                       text=True, timeout=110)
    print(p.stdout[-3000:])
    assert p.returncode == 0 and "CAPTURE_OK" in p.stdout
