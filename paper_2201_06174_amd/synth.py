"""Seeded synthetic seismic volumes and stencils (inputs only).

The paper evaluates on two real SEG-Y surveys (F3 North Sea, Great South
Basin; Sec. 3) that are not available here.  These generators stand in for
them with layered-earth volumes of the same kind: a 1D random reflectivity
(laterally constant layers), optional sinuous channels and a salt body,
planar normal faults that cut everything, a 25 Hz Ricker wavelet along time
and white noise at a fixed SNR.

This module holds none of the saliency method's arithmetic; it only builds
inputs (volumes, structure masks, stencil offset lists, loss weights), and is
shared by the tests, the benchmark and the smoke check.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np

DT = 0.004          # sample interval, s
RICKER_HZ = 25.0    # wavelet peak frequency
RICKER_TAPS = 41    # +-80 ms


def axis_stencil(d: int) -> np.ndarray:
    """6 directional neighbours at offset d along t, il and xl."""
    o = []
    for a in range(3):
        for sgn in (-1, 1):
            v = [0, 0, 0]
            v[a] = sgn * d
            o.append(v)
    return np.array(o, np.int32)


def cube_stencil(d: int) -> np.ndarray:
    """26 neighbours {-d, 0, d}^3 without the centre."""
    o = [[a, b, c] for a in (-d, 0, d) for b in (-d, 0, d) for c in (-d, 0, d) if (a, b, c) != (0, 0, 0)]
    return np.array(o, np.int32)


def ricker(f: float = RICKER_HZ, dt: float = DT, taps: int = RICKER_TAPS) -> np.ndarray:
    t = (np.arange(taps) - taps // 2) * dt
    a = (np.pi * f * t) ** 2
    return ((1.0 - 2.0 * a) * np.exp(-a)).astype(np.float64)


@dataclass
class Fault:
    strike_deg: float   # direction of the fault trace in the (il, xl) plane, from the il axis
    dip_deg: float      # dip from horizontal, in voxel units
    throw: int          # vertical slip of the hanging wall, samples
    centre: Tuple[float, float, float]


@dataclass
class VolumeSpec:
    shape: Tuple[int, int, int]
    faults: List[Fault] = field(default_factory=list)
    channels: int = 0
    salt: Optional[Tuple[Tuple[float, float, float], Tuple[float, float, float]]] = None  # (centre, semi-axes)
    snr_db: float = 10.0


def _layered_reflectivity(rng, length: int) -> np.ndarray:
    r = np.zeros(length, np.float64)
    t = int(rng.integers(3, 13))
    while t < length:
        r[t] = rng.normal(0.0, 0.1)
        t += int(rng.integers(3, 13))
    return r


def _fault_geometry(f: Fault, shape, margin):
    T, IL, XL = shape
    tt = np.arange(-margin, T + margin, dtype=np.float64)[:, None, None]
    ii = np.arange(IL, dtype=np.float64)[None, :, None]
    xx = np.arange(XL, dtype=np.float64)[None, None, :]
    phi = np.deg2rad(f.strike_deg)
    # horizontal unit vector perpendicular to the strike (the dip direction)
    di, dx = -np.sin(phi), np.cos(phi)
    u = (ii - f.centre[1]) * di + (xx - f.centre[2]) * dx
    plane_t = f.centre[0] + np.tan(np.deg2rad(f.dip_deg)) * u
    return tt, plane_t


def make_volume(spec: VolumeSpec, seed: int, with_mask: bool = False):
    """Return V float32 [T][IL][XL] (and the uint8 structure mask if asked)."""
    rng = np.random.default_rng(seed)
    T, IL, XL = spec.shape
    margin = RICKER_TAPS // 2 + 16
    Tm = T + 2 * margin
    r1 = _layered_reflectivity(rng, Tm)
    refl = np.broadcast_to(r1[:, None, None], (Tm, IL, XL)).astype(np.float32)
    mask = np.zeros((Tm, IL, XL), np.uint8) if with_mask else None
    for _ in range(spec.channels):
        t_ch = int(rng.integers(margin + T // 8, margin + (7 * T) // 8))
        x0 = rng.uniform(0.25 * XL, 0.75 * XL)
        A = rng.uniform(20.0, 60.0)
        lam = rng.uniform(100.0, 300.0)
        ph = rng.uniform(0.0, 2 * np.pi)
        width = int(rng.integers(4, 9))
        il = np.arange(IL, dtype=np.float64)
        centre = x0 + A * np.sin(2 * np.pi * il / lam + ph)
        inside = np.abs(np.arange(XL)[None, :] - centre[:, None]) < width / 2.0
        refl[t_ch:t_ch + 2][:, inside] += np.float32(-0.3)
        if with_mask:
            mask[t_ch:t_ch + 2][:, inside] = 1
    if spec.salt is not None:
        (ct, ci, cx), (at, ai, ax) = spec.salt
        ii = np.arange(IL, dtype=np.float64)[:, None]
        xx = np.arange(XL, dtype=np.float64)[None, :]
        ri, rx = ((ii - ci) / ai) ** 2, ((xx - cx) / ax) ** 2
        # one t plane at a time (the same arithmetic and the same draw order as the whole
        # volume at once: the interior's normal draws follow C order, plane after plane)
        for k in range(Tm):
            rt = ((k - margin - ct) / at) ** 2
            if rt > (1.0 + 1.0 / at) ** 2:
                continue  # the plane misses the body and its shell
            rho = np.sqrt(rt + ri + rx)
            shell = np.abs(rho - 1.0) < 1.0 / at
            interior = (rho < 1.0) & ~shell
            plane = refl[k]
            plane[interior] = rng.normal(0.0, 0.05, size=int(interior.sum())).astype(np.float32)
            plane[shell] = np.float32(0.5)
            if with_mask:
                mask[k][shell] = 1
    for f in spec.faults:
        tt, plane_t = _fault_geometry(f, spec.shape, margin)
        hanging = tt < plane_t          # above the plane (shallower)
        src = np.roll(refl, f.throw, axis=0)   # value from t - throw
        refl = np.where(hanging, src, refl)
        if with_mask:
            mask = np.where(hanging, np.roll(mask, f.throw, axis=0), mask)
            near = np.abs(tt - plane_t) * np.cos(np.deg2rad(f.dip_deg)) <= 2.0
            mask = np.where(near, np.uint8(1), mask)
        del tt, plane_t, hanging, src
    from scipy.ndimage import convolve1d
    sig = convolve1d(refl, ricker().astype(np.float32), axis=0, mode="constant")
    sig = np.ascontiguousarray(sig[margin:margin + T])
    p = float(np.mean(sig.astype(np.float64) ** 2))
    sigma = np.sqrt(p / (10.0 ** (spec.snr_db / 10.0))) if p > 0 else 0.0
    noise = rng.standard_normal(size=sig.shape, dtype=np.float32) * np.float32(sigma)
    V = (sig + noise).astype(np.float32)
    if with_mask:
        return V, np.ascontiguousarray(mask[margin:margin + T])
    return V


def centre_fault(shape, throw=6, dip=60.0) -> Fault:
    T, IL, XL = shape
    return Fault(strike_deg=0.0, dip_deg=dip, throw=throw, centre=((T - 1) / 2.0, (IL - 1) / 2.0, (XL - 1) / 2.0))


def random_faults(rng, shape, count) -> List[Fault]:
    T, IL, XL = shape
    out = []
    for _ in range(count):
        out.append(Fault(strike_deg=rng.uniform(0.0, 180.0), dip_deg=rng.uniform(45.0, 75.0),
                         throw=int(rng.integers(3, 11)),
                         centre=(rng.uniform(0.2, 0.8) * T, rng.uniform(0.2, 0.8) * IL, rng.uniform(0.2, 0.8) * XL)))
    return out


@dataclass
class Workload:
    """One named workload: volume recipe plus the method's parameters."""
    name: str
    spec: VolumeSpec
    seed: int
    n: int
    s: int
    offsets: np.ndarray
    window: str = "hann"


def workload(name: str, idx: int = 0) -> Workload:
    """The five workloads: small (64^3), survey (256x400x600), salt (512^3),
    batch member idx (uneven subvolume), grad (128^3)."""
    if name == "small":
        shape = (64, 64, 64)
        return Workload(name, VolumeSpec(shape, faults=[centre_fault(shape)]), 1000 * 1 + idx, 8, 1, axis_stencil(4))
    if name == "survey":
        shape = (256, 400, 600)
        rng = np.random.default_rng(1000 * 2 + 500 + idx)
        return Workload(name, VolumeSpec(shape, faults=random_faults(rng, shape, 5), channels=2), 1000 * 2 + idx, 16, 2,
                        cube_stencil(8))
    if name == "salt":
        shape = (512, 512, 512)
        return Workload(name, VolumeSpec(shape, salt=((300.0, 256.0, 256.0), (120.0, 150.0, 150.0))), 1000 * 3 + idx,
                        16, 2, cube_stencil(8))
    if name == "batch":
        rng = np.random.default_rng(1000 * 4 + 500)
        sizes = rng.integers(32, 161, size=(96, 3))
        ns = rng.choice(np.array([8, 12, 16]), size=96)
        shape = tuple(int(v) for v in sizes[idx])
        n = int(ns[idx])
        s = 1 if n == 8 else 2
        return Workload("batch%d" % idx, VolumeSpec(shape, faults=[centre_fault(shape)]), 1000 * 4 + idx, n, s,
                        axis_stencil(n // 2))
    if name == "grad":
        shape = (128, 128, 128)
        return Workload(name, VolumeSpec(shape, faults=[centre_fault(shape)]), 1000 * 5 + idx, 8, 1, axis_stencil(4))
    raise KeyError(name)


def loss_weights(shape, seed: int = 5001) -> np.ndarray:
    """U(0,1) weights of the scalar loss sum(S * weights)."""
    return np.random.default_rng(seed).uniform(0.0, 1.0, size=shape).astype(np.float32)


def grid_shape(shape, s):
    return tuple(-(-int(N) // int(s)) for N in shape)


def desired_map(mask_full: np.ndarray, s: int):
    """Desired map D on the grid (structure mask at the centres) and the fit
    mask selecting the middle inline section of the grid."""
    D = np.ascontiguousarray(mask_full[::s, ::s, ::s]).astype(np.float32)
    M = np.zeros(D.shape, np.uint8)
    M[:, D.shape[1] // 2, :] = 1
    return D, M
