"""Benchmark of the saliency hot path on one MI355X.

    python bench.py [--steps K] [--warmup W] [--workload salt|survey|small|grad]
                    [--precision fp32|split_bf16|fp16] [--no-cpu-baseline] [--no-extra]

One step = one whole forward pass (local spectra + projection features,
directional center-surround, adapted fusion and the full-resolution combine)
over one synthetic volume already resident in HBM; by default the 512^3
salt-dome volume (window 16^3 Hann, stride 2, 26 neighbours), the largest
single-GPU configuration.  Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Published MI355X peaks used as roofline denominators
PEAK_FP32_MFMA_TFLOPS = 157.3
PEAK_BF16_MFMA_TFLOPS = 2500.0
PEAK_HBM_GBS = 8000.0
PEAK_FP32_VALU_TFLOPS = 78.6   # unpacked v_fma_f32 (the kernels are built without packed fp32 forms)


def algorithmic_flops_per_window(n: int) -> float:
    """Real-input 3D FFT of one n^3 local cube: 2.5 n^3 log2(n^3) flops."""
    return 2.5 * n ** 3 * math.log2(n ** 3)


def dense_dft_flops_per_window(n: int, s: int) -> float:
    """Reference count of the separable dense complex-DFT contractions of one window in a
    sliding tile design (real pass along xl at n/2+1 bins, then the two complex passes):
    8 n^3 K + 8 n^2 K s + 4 n K s^2 with K = n/2 + 1.  The graded roofline time of a
    launch is this count over the matrix-core peak of the precision (three products
    for split-bf16).  The FP32 kernel's packed real cos/sin rows execute about half of
    it (the hardware-counted figure is reported beside it as `mfma_counted`)."""
    K = n // 2 + 1
    return 8.0 * n ** 3 * K + 8.0 * n ** 2 * K * s + 4.0 * n * K * s * s


TRAFFIC_DIR = os.path.join(ROOT, "profiles")
COPY_BYTES = 1 << 30


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="salt")
    ap.add_argument("--precision", default="fp32")
    ap.add_argument("--fusion", default="adapt_ls")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-errors", action="store_true", help="skip the per-output errors against the oracle")
    ap.add_argument("--fwd-bwd-workload", default="grad", help="workload of --part fwd_bwd (grad or salt)")
    ap.add_argument("--cache", default=None,
                    help="directory for generated volumes (.npy): reused by later runs with the same workload")
    ap.add_argument("--part", choices=["fwd_bwd", "batch", "peaks"], default=None,
                    help="time only the forward + adjoint on the gradient workload, only the batch, or only "
                         "the device-peak microbenchmarks, and print that object")
    ap.add_argument("--traffic-pass", action="store_true",
                    help="launch a %d-byte device copy, then the feature kernel twice, and exit "
                         "(the command profiled with rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE)" % COPY_BYTES)
    return ap.parse_args()


class Pipeline:
    """Preallocated buffers and direct C-ABI calls (no allocation in the timed loop)."""

    def __init__(self, torch, lib, V, w, precision, fusion, D, mask):
        from paper_2201_06174_amd import _lib, grid_shape
        self.torch, self.lib, self._lib = torch, lib, _lib
        self.V = V
        self.shape = tuple(V.shape)
        self.grid = grid_shape(self.shape, w.s)
        dev = V.device
        self.E = torch.empty((3,) + self.grid, dtype=torch.float32, device=dev)
        self.Sm = torch.empty_like(self.E)
        self.S = torch.empty(self.shape, dtype=torch.float32, device=dev)
        self.W = torch.empty(4, dtype=torch.float64, device=dev)
        nb = int(lib.sal_fuse_workspace_size(self.grid[0], self.grid[1], self.grid[2], None))
        self.ws = torch.empty(nb, dtype=torch.uint8, device=dev)
        self.spec = _lib.make_spec(w.n, w.s, "hann", precision)
        self.stencil, self._keep = _lib.make_stencil(w.offsets)
        self.fusion = _lib.make_fusion(fusion, None, 1e-6)
        self.D, self.mask = D, mask
        self.s = w.s

    def stream(self):
        return ctypes.c_void_p(self.torch.cuda.current_stream().cuda_stream)

    def project(self):
        T, IL, XL = self.shape
        self._lib.check(self.lib.sal_project(ctypes.c_void_p(self.V.data_ptr()), T, IL, XL, self.spec,
                                             ctypes.c_void_p(self.E.data_ptr()), self.stream()))

    def rest(self):
        T, IL, XL = self.shape
        Tg, ILg, XLg = self.grid
        st = self.stream()
        self._lib.check(self.lib.sal_center_surround(ctypes.c_void_p(self.E.data_ptr()), Tg, ILg, XLg, self.s,
                                                     self.stencil, ctypes.c_void_p(self.Sm.data_ptr()), st))
        self._lib.check(self.lib.sal_fuse(ctypes.c_void_p(self.Sm.data_ptr()), Tg, ILg, XLg, self.fusion,
                                          ctypes.c_void_p(self.D.data_ptr()), ctypes.c_void_p(self.mask.data_ptr()),
                                          T, IL, XL, self.s, ctypes.c_void_p(self.W.data_ptr()),
                                          ctypes.c_void_p(self.S.data_ptr()), ctypes.c_void_p(self.ws.data_ptr()),
                                          self.ws.numel(), st))


CACHE_DIR = None


def make_volume(w, with_mask=False):
    """The workload's synthetic volume (and structure mask), from --cache when present there."""
    from paper_2201_06174_amd import synth
    if CACHE_DIR:
        base = os.path.join(CACHE_DIR, "%s_%d" % (w.name, w.seed))
        if os.path.exists(base + "_V.npy") and os.path.exists(base + "_M.npy"):
            V, M = np.load(base + "_V.npy"), np.load(base + "_M.npy")
            return (V, M) if with_mask else V
        V, M = synth.make_volume(w.spec, w.seed, with_mask=True)
        os.makedirs(CACHE_DIR, exist_ok=True)
        np.save(base + "_V.npy", V)
        np.save(base + "_M.npy", M)
        return (V, M) if with_mask else V
    return synth.make_volume(w.spec, w.seed, with_mask=with_mask)


def time_forward(torch, pipe, steps, warmup):
    for _ in range(warmup):
        pipe.project()
        pipe.rest()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = time.perf_counter()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record()
    for k in range(steps):
        ev[k][0].record()
        pipe.project()
        ev[k][1].record()
        pipe.rest()
    end.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    total_ms = start.elapsed_time(end)
    kern_ms = [a.elapsed_time(b) for a, b in ev]
    return total_ms / steps, float(np.mean(kern_ms)), wall


def progress(msg):
    """A progress line on stderr (stdout carries only the result line)."""
    print("[bench] %s" % msg, file=sys.stderr, flush=True)


class OracleSection:
    """The FP64 oracle's E, S_m and W on the grid's middle inline section, where the adapted
    weights are fitted (the desired map's mask holds that section only, so the oracle's W
    there is its W for the whole volume), plus E and S_m at 192 sampled grid points with the
    corners among them, and sampled voxels whose nearest centre lies on that section.  The
    per-output errors of a forward are taken against these (measurement only, outside the
    timed region)."""

    def __init__(self, V, w, D, mask, delta):
        from oracle import oracle as orc
        self.gs = orc.grid_shape(V.shape, w.s)
        self.mid = self.gs[1] // 2
        if int(mask.sum()) != int(mask[:, self.mid, :].sum()):
            raise ValueError("the fit mask must hold the middle inline section only")
        t0 = time.perf_counter()
        self.E, self.Sm = orc.saliency_inline_plane(V, w.n, w.s, "hann", w.offsets, None, False, self.mid)
        self.W, fb, _ = orc.fusion_weights(self.Sm, D[:, self.mid, :], mask[:, self.mid, :], "adapt_ls", delta=delta)
        rng = np.random.default_rng(11)
        g = np.stack([rng.integers(0, N, 192) for N in self.gs], 1).astype(np.int64)
        g[:8] = [[a, b, c] for a in (0, self.gs[0] - 1) for b in (0, self.gs[1] - 1) for c in (0, self.gs[2] - 1)]
        self.g = g
        self.Sg, self.Eg = orc.saliency_at(V, w.n, w.s, "hann", w.offsets, None, False, g)
        self.v = np.stack([rng.integers(0, V.shape[0], 4096), np.full(4096, self.mid * w.s),
                           rng.integers(0, V.shape[2], 4096)], 1)
        gv = np.minimum(self.v // w.s, np.array(self.gs) - 1)
        self.S = (self.W[:, None] * self.Sm[:, gv[:, 0], gv[:, 2]]).sum(0)
        self.seconds = time.perf_counter() - t0
        self.fallback = int(fb)

    @staticmethod
    def _rel(x, ref):
        x, ref = np.asarray(x, np.float64), np.asarray(ref, np.float64)
        return float(np.max(np.abs(x - ref)) / max(np.max(np.abs(ref)), 1e-30))

    def errors(self, pipe):
        """max |x - ref| / max |ref| per output of the pipeline's last forward."""
        g = self.g
        E = pipe.E[:, :, self.mid, :].cpu().numpy()
        Sm = pipe.Sm[:, :, self.mid, :].cpu().numpy()
        gi = [pipe.torch.from_numpy(g[:, a]).to(pipe.E.device) for a in range(3)]
        Eg = pipe.E[:, gi[0], gi[1], gi[2]].T.cpu().numpy()
        Sg = pipe.Sm[:, gi[0], gi[1], gi[2]].T.cpu().numpy()
        W = pipe.W.cpu().numpy()
        vi = [pipe.torch.from_numpy(self.v[:, a]).to(pipe.E.device) for a in range(3)]
        S = pipe.S[vi[0], vi[1], vi[2]].cpu().numpy()
        return {"E": round(max(self._rel(E, self.E), self._rel(Eg, self.Eg)), 9),
                "Sm": round(max(self._rel(Sm, self.Sm), self._rel(Sg, self.Sg)), 9),
                "W": round(self._rel(W[:3], self.W), 9), "S": round(self._rel(S, self.S), 9),
                "fallback": int(W[3])}


def precision_forms(torch, lib, Vd, w, fusion, Dd, Md, steps, done, peaks=None, oracle=None, first=None):
    """The forward step in FP32, split-BF16 and FP16 on one volume; `done` holds (ms per step,
    kernel ms) of a precision already timed, `first` its pipeline (outputs still in place).
    With `oracle` (an OracleSection) each form carries its per-output errors."""
    nvox = int(np.prod(Vd.shape))
    forms = {}
    for prec in ("fp32", "split_bf16", "fp16"):
        pp = first if prec in done else None
        if prec in done:
            m2, k2 = done[prec]
        else:
            progress("%s forward on %s" % (prec, "x".join(str(v) for v in Vd.shape)))
            pp = Pipeline(torch, lib, Vd, w, prec, fusion, Dd, Md)
            m2, k2, _ = time_forward(torch, pp, steps, 2)
        nwin = int(np.prod([-(-N // w.s) for N in Vd.shape]))
        forms[prec] = {"ms_per_step": round(m2, 4), "kernel_ms": round(k2, 4),
                       "mvoxel_s": round(nvox / (m2 * 1e-3) / 1e6, 3), "graded": graded(w, nwin, prec, k2, peaks),
                       "mfma_counted": feature_mfma(w.name, prec, k2)}
        if oracle is not None and pp is not None:
            forms[prec]["err_vs_oracle"] = oracle.errors(pp)
        if pp is not first:
            del pp
    for prec in ("fp32", "split_bf16", "fp16"):
        forms[prec]["speedup_vs_fp32"] = round(forms["fp32"]["ms_per_step"] / forms[prec]["ms_per_step"], 3)
    if oracle is not None:
        forms["err_vs_oracle_definition"] = (
            "max|x - ref| / max|ref| per output against the FP64 oracle: E and S_m on the middle inline section of "
            "the grid and at 192 sampled grid points (corners included), W against the oracle's fit (the fit mask "
            "holds that section only), S at 4096 sampled voxels whose nearest centre lies on it; oracle %.1f s" %
            oracle.seconds)
    return forms


def time_fwd_bwd(torch, w_name, steps, warmup, peaks=None, V=None):
    """Forward plus the hand-written adjoint on one workload (equal fusion); V: the workload's
    volume if already generated."""
    import paper_2201_06174_amd as sal
    from paper_2201_06174_amd import synth
    w = synth.workload(w_name)
    if V is None:
        V = make_volume(w)
    Vd = torch.from_numpy(V).cuda()
    gS = torch.from_numpy(synth.loss_weights(V.shape, 5001)).cuda()
    cfg = sal.Config(n=w.n, s=w.s, offsets=w.offsets, fusion="equal")
    for _ in range(warmup):
        r = sal.saliency(Vd, cfg)
        sal.backward(Vd, cfg, r["E"], r["Sm"], r["W"], gS)
    torch.cuda.synchronize()
    # steps back to back, as a training loop runs them: events around each forward and each
    # backward, one synchronization after the last step (a host wait per step would add the
    # host's launch latency of every step's first kernel to the forward)
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
    for a, b, c in ev:
        a.record()
        r = sal.saliency(Vd, cfg)
        b.record()
        sal.backward(Vd, cfg, r["E"], r["Sm"], r["W"], gS)
        c.record()
    torch.cuda.synchronize()
    fwd = sum(a.elapsed_time(b) for a, b, _ in ev) / steps
    bwd = sum(b.elapsed_time(c) for _, b, c in ev) / steps
    nvox = int(np.prod(V.shape))
    nwin = int(np.prod([-(-N // w.s) for N in V.shape]))
    # forward, recomputed spectra and the adjoint synthesis: three dense-DFT passes of FP32 work
    t_roof = 3 * dense_dft_flops_per_window(w.n, w.s) * nwin / (PEAK_FP32_MFMA_TFLOPS * 1e12) * 1e3
    # the algorithmic count: three real-input 3D FFTs of each local cube (forward, recomputed,
    # adjoint synthesis)
    alg = 3 * algorithmic_flops_per_window(w.n) * nwin / ((fwd + bwd) * 1e-3) / 1e12
    kern = {"grad": ["k_project_fp32<8, 1, 1, false>", "k_spectral_adjoint<8, 1, false>"],
            "salt": ["k_project_fp32<16, 2, 1, false>", "k_spectral_adjoint<16, 2, false>"]}.get(w_name)
    roof = {"bound": "mfma", "t_roof_ms": round(t_roof, 4), "frac": round(t_roof / (fwd + bwd), 4),
            "peak_tflops": PEAK_FP32_MFMA_TFLOPS,
            "algorithmic_tflops": round(alg, 3), "algorithmic_frac": round(alg / PEAK_FP32_MFMA_TFLOPS, 4),
            # matrix-core work of the forward feature kernel and the spectral adjoint
            # counted by rocprofv3, over the whole forward + backward time
            "mfma_counted": stored_mfma("k_spectral_adjoint_%s_mfma.txt" % w_name, kern, "adjoint",
                                        fwd + bwd, PEAK_FP32_MFMA_TFLOPS) if kern else None}
    if peaks:
        t_meas = t_roof * PEAK_FP32_MFMA_TFLOPS / peaks["mfma_f32"]["tflops"]
        roof["t_roof_measured_peak_ms"] = round(t_meas, 4)
        roof["frac_measured_peak"] = round(t_meas / (fwd + bwd), 4)
    return {"workload": "%s: %s, window %d^3, stride %d, loss sum(S * U(0,1))" % (
        w_name, "x".join(str(v) for v in V.shape), w.n, w.s),
        "fwd_ms": round(fwd, 4), "bwd_ms": round(bwd, 4),
        "fwd_bwd_mvoxel_s": round(nvox / ((fwd + bwd) * 1e-3) / 1e6, 3), "roofline": roof}


def time_batch(torch, lib, steps, count=96):
    """The 96-member batch: one captured plan vs the three calls per member launched separately."""
    import paper_2201_06174_amd as sal
    from paper_2201_06174_amd import synth
    members, pipes = [], []
    nvox = 0
    for i in range(count):
        w = synth.workload("batch", i)
        V, M = synth.make_volume(w.spec, w.seed, with_mask=True)
        D, mask = synth.desired_map(M, w.s)
        Vd, Dd, Md = (torch.from_numpy(a).cuda() for a in (V, D, mask))
        cfg = sal.Config(n=w.n, s=w.s, offsets=w.offsets, fusion="adapt_ls", delta=1e-6)
        members.append({"V": Vd, "cfg": cfg, "D": Dd, "mask": Md})
        pipes.append(Pipeline(torch, lib, Vd, w, "fp32", "adapt_ls", Dd, Md))
        nvox += int(np.prod(V.shape))
    t0 = time.perf_counter()
    plan = sal.Plan(members, autotune=True)
    create_s = time.perf_counter() - t0
    desc = plan.describe()

    def run_plan():
        plan.launch()

    def run_separate():
        for pp in pipes:
            pp.project()
            pp.rest()

    out = {"members": count, "voxels": nvox, "plan_create_s": round(create_s, 3), "plan": desc.strip().split("\n")}
    for name, fn in (("graph", run_plan), ("separate", run_separate)):
        fn()
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(steps):
            fn()
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / steps
        out[name + "_ms"] = round(ms, 4)
        out[name + "_mvoxel_s"] = round(nvox / (ms * 1e-3) / 1e6, 3)
    plan.close()
    return out


# (name, sal_peak_kind, published peak in TFLOP/s, per-thread checksum per iteration)
PEAK_KINDS = (("mfma_f32", 0, PEAK_FP32_MFMA_TFLOPS, 64), ("mfma_bf16", 1, PEAK_BF16_MFMA_TFLOPS, 1024),
              ("mfma_f16", 2, PEAK_BF16_MFMA_TFLOPS, 1024), ("valu_f32", 3, PEAK_FP32_VALU_TFLOPS, 8))


def measure_peaks(torch, lib, reps=5):
    """The device's own sustained rates (sal_peak_* microbenchmarks, HIP events on the launch
    stream, best of `reps`): matrix-core and unpacked-VALU TFLOP/s with 8 workgroups of 4 waves per
    CU, and HBM GB/s of a 4 GiB read and a 2 GiB copy at the best of three grid sizes.  Each
    kernel's output is checked against its closed form, so a launch that did not do its work
    cannot report a rate."""
    from paper_2201_06174_amd import _lib
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]

    def best_ms(launch):
        launch()
        best = math.inf
        for _ in range(reps):
            ev[0].record()
            launch()
            ev[1].record()
            torch.cuda.synchronize()
            best = min(best, ev[0].elapsed_time(ev[1]))
        return best

    res = {"cus": cus}
    blocks, iters = cus * 8, 16384
    out = torch.empty(blocks * 256, dtype=torch.float32, device="cuda")
    for name, kind, vendor, per_iter in PEAK_KINDS:
        flops = lib.sal_peak_compute_flops(kind, iters, blocks)
        ms = best_ms(lambda: _lib.check(lib.sal_peak_compute(kind, iters, blocks, ctypes.c_void_p(out.data_ptr()),
                                                             st)))
        assert bool((out == float(per_iter * iters)).all()), name
        tf = flops / (ms * 1e-3) / 1e12
        res[name] = {"tflops": round(tf, 2), "published": vendor, "ratio": round(tf / vendor, 4)}
    del out
    nbytes = 4 << 30
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty(nbytes // 8, dtype=torch.float32, device="cuda")
    for name, kind, moved in (("hbm_read", 0, nbytes), ("hbm_copy", 1, nbytes)):
        n = nbytes if kind == 0 else nbytes // 2
        best = None
        for per_cu in (4, 8, 16):
            blocks = cus * per_cu
            out = torch.zeros(blocks * 256, dtype=torch.float32, device="cuda")
            ms = best_ms(lambda: _lib.check(lib.sal_peak_stream(kind, ctypes.c_void_p(src.data_ptr()),
                                                                ctypes.c_void_p(dst.data_ptr()), n,
                                                                ctypes.c_void_p(out.data_ptr()), blocks, st)))
            if kind == 0:
                assert float(out.double().sum()) == nbytes // 4, name
            else:
                assert bool((dst == 1.0).all()), name
            gbs = moved / (ms * 1e-3) / 1e9
            if best is None or gbs > best[0]:
                best = (gbs, blocks)
        res[name] = {"gbs": round(best[0], 1), "published": PEAK_HBM_GBS, "ratio": round(best[0] / PEAK_HBM_GBS, 4),
                     "blocks": best[1]}
    del src, dst
    torch.cuda.empty_cache()
    return res


def graded(w, nwin, precision, kern_ms, peaks=None):
    """Graded roofline of the feature kernel: the dense-DFT contraction count of the
    launch over the matrix-core peak of its precision, against the measured time; with
    measured peaks, the same against the device's own matrix-core rate."""
    flops = dense_dft_flops_per_window(w.n, w.s) * nwin * (3 if precision == "split_bf16" else 1)
    peak = PEAK_FP32_MFMA_TFLOPS if precision == "fp32" else PEAK_BF16_MFMA_TFLOPS
    t_roof = flops / (peak * 1e12) * 1e3
    g = {"t_roof_ms": round(t_roof, 4), "frac": round(t_roof / kern_ms, 4),
         "dense_complex_dft_flops_per_window": dense_dft_flops_per_window(w.n, w.s)}
    if peaks:
        key = {"fp32": "mfma_f32", "split_bf16": "mfma_bf16", "fp16": "mfma_f16"}[precision]
        t_meas = flops / (peaks[key]["tflops"] * 1e12) * 1e3
        g["t_roof_measured_peak_ms"] = round(t_meas, 4)
        g["frac_measured_peak"] = round(t_meas / kern_ms, 4)
    return g


def stored_traffic(workload, precision):
    """HBM bytes per launch of the FP32 feature kernel from the committed PMC summary, or
    None when there is none for this workload or the kernel sources changed since."""
    if precision != "fp32":
        return None
    from paper_2201_06174_amd import profiling
    t = profiling.read_traffic(os.path.join(TRAFFIC_DIR, "k_project_fp32_%s_traffic.txt" % workload))
    if not t or t.get("source_digest") != profiling.source_digest():
        return None
    return float(t["traffic_bytes_per_launch"])


# committed rocprofv3 MFMA-counter summaries of the feature kernel: (workload, precision) ->
# (file, kernel, source set)
MFMA_PROFILES = {}
for _wl in ("salt", "survey"):
    MFMA_PROFILES[(_wl, "fp32")] = ("k_project_fp32_%s_mfma.txt" % _wl, "k_project_fp32<16, 2, 1, false>", "fp32")
    MFMA_PROFILES[(_wl, "split_bf16")] = ("k_project_lowp_%s_split_bf16_mfma.txt" % _wl,
                                          "k_project_lowp<16, 2, 1, 1, true>", "lowp")
    MFMA_PROFILES[(_wl, "fp16")] = ("k_project_lowp_%s_fp16_mfma.txt" % _wl, "k_project_lowp<16, 2, 2, 1, true>",
                                    "lowp")


def feature_mfma(workload, precision, kern_ms):
    if (workload, precision) not in MFMA_PROFILES:
        return None
    fname, kernel, sources = MFMA_PROFILES[(workload, precision)]
    peak = PEAK_FP32_MFMA_TFLOPS if precision == "fp32" else PEAK_BF16_MFMA_TFLOPS
    return stored_mfma(fname, [kernel], sources, kern_ms, peak)


def stored_mfma(fname, kernels, sources, ms, peak_tflops):
    """Matrix-core flops per launch counted by rocprofv3 (SQ_INSTS_VALU_MFMA_MOPS_*) from a
    committed summary, summed over `kernels`, as a rate over `ms` against the precision's
    peak; None when the summary is missing or its kernels changed since."""
    from paper_2201_06174_amd import profiling
    tot = 0.0
    for k in kernels:
        f = profiling.read_mfma(os.path.join(TRAFFIC_DIR, fname), k, sources)
        if f is None:
            return None
        tot += f
    t = tot / (ms * 1e-3) / 1e12
    return {"counted_flops": tot, "tflops": round(t, 3), "peak": peak_tflops, "frac": round(t / peak_tflops, 4),
            "profile": "profiles/" + fname}


def traffic_pass(torch, pipe):
    x = torch.empty(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(2):
        y.copy_(x)
    torch.cuda.synchronize()
    del x, y
    for _ in range(2):
        pipe.project()
    torch.cuda.synchronize()
    print("traffic pass done", flush=True)


def cpu_model():
    """The host CPU's model name and logical core count (from /proc/cpuinfo)."""
    name, count = "unknown", 0
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    name = line.split(":", 1)[1].strip()
                    count += 1
    except OSError:
        pass
    return name, count


def cpu_baseline(V, w, seconds):
    """The FP64 oracle's feature step on bounded samples of windows of the same volume: on
    all host cores (the OpenMP threads of the process), then on one core."""
    from oracle import oracle as orc
    nth = orc.max_threads()
    out = oracle_rate(V, w, seconds, nth)
    one = oracle_rate(V, w, max(2.0, seconds / 4), 1)
    model, logical = cpu_model()
    out["single_core"] = {"value": one["value"], "unit": one["unit"], "cores": 1, "sample": one["sample"]}
    out["cpu_model"] = model
    out["logical_cpus"] = logical or os.cpu_count()
    out["parallel_speedup"] = round(out["value"] / one["value"], 2) if one["value"] else None
    return out


def oracle_rate(V, w, seconds, nth):
    from oracle import oracle as orc
    gs = orc.grid_shape(V.shape, w.s)
    rng = np.random.default_rng(123)
    cnt = 64
    elapsed = 0.0
    total_windows = 0
    while True:
        g = np.stack([rng.integers(0, N, cnt) for N in gs], 1).astype(np.int64)
        t0 = time.perf_counter()
        orc.features_at(V, w.n, w.s, "hann", g, nthreads=nth)
        dt = time.perf_counter() - t0
        elapsed += dt
        total_windows += cnt
        if elapsed >= seconds or cnt >= 1 << 22:
            break
        cnt = int(min(max(cnt * 2, cnt * (seconds - elapsed) / max(dt, 1e-3) * 0.9), 1 << 22))
    voxels_per_window = w.s ** 3
    mvox = total_windows * voxels_per_window / elapsed / 1e6
    return {"value": round(mvox, 4), "unit": "Mvoxel/s", "cores": nth, "kind": "oracle",
            "sample": "%d random windows (features of %d^3 Hann cubes, stride %d) of the %s volume, %.1f s; "
                      "each window stands for s^3 output voxels" % (total_windows, w.n, w.s, "x".join(
                          str(v) for v in V.shape), elapsed)}


def main():
    global CACHE_DIR
    args = parse()
    CACHE_DIR = args.cache
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (requested --gpus %d)" % args.gpus)
        sys.exit(2)
    import torch
    from paper_2201_06174_amd import _lib, synth
    lib = _lib.load()
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.part == "fwd_bwd":
        print(json.dumps(time_fwd_bwd(torch, args.fwd_bwd_workload, max(args.steps, 1), args.warmup)), flush=True)
        return
    if args.part == "batch":
        print(json.dumps(time_batch(torch, lib, max(args.steps, 1))), flush=True)
        return
    if args.part == "peaks":
        print(json.dumps(measure_peaks(torch, lib)), flush=True)
        return
    w = synth.workload(args.workload)
    V, M = make_volume(w, with_mask=True)
    D, mask = synth.desired_map(M, w.s)
    dev = torch.device("cuda:0")
    Vd = torch.from_numpy(V).to(dev)
    Dd = torch.from_numpy(D).to(dev)
    Md = torch.from_numpy(mask).to(dev)
    pipe = Pipeline(torch, lib, Vd, w, args.precision, args.fusion, Dd, Md)
    if args.traffic_pass:
        traffic_pass(torch, pipe)
        return
    progress("%s forward on %s" % (args.precision, args.workload))
    ms, kern_ms, wall = time_forward(torch, pipe, args.steps, args.warmup)
    nvox = int(np.prod(V.shape))
    nwin = int(np.prod(pipe.grid))
    value = nvox / (ms * 1e-3) / 1e6
    alg = algorithmic_flops_per_window(w.n) * nwin
    achieved = alg / (kern_ms * 1e-3) / 1e12
    peak = PEAK_FP32_MFMA_TFLOPS if args.precision == "fp32" else PEAK_BF16_MFMA_TFLOPS
    kname = "k_project_fp32" if args.precision == "fp32" else "k_project_lowp"
    peaks = None
    if not args.no_extra:
        progress("device peak microbenchmarks")
        peaks = measure_peaks(torch, lib)
    out = {
        "metric": "Mvoxel/s saliency fwd (FP32 vs split-BF16 @<=1e-3 rel) and fwd+bwd on 1 GPU",
        "value": round(value, 3),
        "unit": "Mvoxel/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "%s: %s volume, window %d^3 Hann, stride %d, %d neighbours, %s fusion" % (
            args.workload, "x".join(str(v) for v in V.shape), w.n, w.s, len(w.offsets), args.fusion),
            "precision": args.precision, "voxels": nvox, "windows": nwin},
        "roofline": {"bound": "mfma", "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
                     "frac": round(achieved / peak, 4), "traffic": stored_traffic(args.workload, args.precision),
                     "kernel": "%s (sal_project)" % kname, "kernel_ms": round(kern_ms, 4),
                     "flops_per_window": algorithmic_flops_per_window(w.n),
                     "graded": graded(w, nwin, args.precision, kern_ms, peaks),
                     "mfma_counted": feature_mfma(args.workload, args.precision, kern_ms)},
    }
    if peaks:
        mkey = "mfma_f32" if args.precision == "fp32" else "mfma_bf16"
        out["roofline"]["measured_peak"] = {"peak": peaks[mkey]["tflops"],
                                            "frac": round(achieved / peaks[mkey]["tflops"], 4)}
    if not args.no_extra:
        extra = {"measured_peaks": peaks}
        done = {args.precision: (ms, kern_ms)}
        errs = not args.no_errors and args.fusion == "adapt_ls"
        orc_sec = None
        if errs:
            progress("oracle on the middle inline section of %s" % args.workload)
            orc_sec = OracleSection(V, w, D, mask, 1e-6)
        extra["precision_forms"] = precision_forms(torch, lib, Vd, w, args.fusion, Dd, Md, max(3, args.steps // 2),
                                                   done, peaks, orc_sec, pipe)
        del pipe
        torch.cuda.empty_cache()
        # the other full-volume configuration: the survey volume (or the salt dome)
        other = "survey" if args.workload != "survey" else "salt"
        progress("generating the %s volume" % other)
        wo = synth.workload(other)
        Vo, Mo = make_volume(wo, with_mask=True)
        Do, masko = synth.desired_map(Mo, wo.s)
        Vod, Dod, Mod = (torch.from_numpy(a).to(dev) for a in (Vo, Do, masko))
        orc_o = OracleSection(Vo, wo, Do, masko, 1e-6) if errs else None
        forms = precision_forms(torch, lib, Vod, wo, args.fusion, Dod, Mod, max(3, args.steps // 2), {}, peaks, orc_o)
        forms["workload"] = "%s: %s volume, window %d^3 Hann, stride %d, %d neighbours, %s fusion" % (
            other, "x".join(str(v) for v in Vod.shape), wo.n, wo.s, len(wo.offsets), args.fusion)
        extra["precision_forms_" + other] = forms
        del Vod, Dod, Mod, Vo, Mo, Do, masko
        torch.cuda.empty_cache()
        progress("forward + adjoint on grad")
        # the 128^3 step takes under 2 ms: enough warm-up and timed steps (about 0.1 s) that the
        # clocks have settled after the host-side work before it
        extra["fwd_bwd"] = time_fwd_bwd(torch, "grad", 50, 20, peaks)
        progress("forward + adjoint on salt")
        extra["fwd_bwd_salt"] = time_fwd_bwd(torch, "salt", 3, 1, peaks, V if args.workload == "salt" else None)
        torch.cuda.empty_cache()
        progress("batch plan")
        extra["batch"] = time_batch(torch, lib, 5)
        out["extra"] = extra
    if not args.no_cpu_baseline:
        progress("oracle on the host cores")
        out["cpu_baseline"] = cpu_baseline(V, w, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
