"""Shared helpers of the gradient parity tests (not collected by pytest).

sgn(E(g) - E(g+o)) decides which way each center-surround term pulls (Eq. 3); where
the oracle's own difference is within a hair of zero the GPU and the oracle may take
different, equally valid subgradients.  Such near-tie terms are found from the
oracle's features, and the voxels their windows reach are the only ones allowed to
differ; the tests bound how many there are."""
import numpy as np

from oracle import oracle as orc


def plane_stencils(offsets, weights, planes):
    """[(offsets, weights)] for the planes t, x, y, weights resolved (Gaussian default)."""
    if planes is not None:
        return [(np.asarray(o), orc.default_weights(o) if w is None else np.asarray(w, np.float64))
                for o, w in planes]
    w = orc.default_weights(offsets) if weights is None else np.asarray(weights, np.float64)
    return [(np.asarray(offsets), w)] * 3


def near_tie_voxels(E, shape, n, s, stencils, literal, tau):
    """Voxels whose gradient involves a center-surround term with |difference| < tau."""
    gs = E.shape[1:]
    amb = np.zeros(gs, bool)
    for m, (off, w) in enumerate(stencils):
        for k, o in enumerate(np.asarray(off) // s):
            sl_a = tuple(slice(max(0, -d), N - max(0, d)) for d, N in zip(o, gs))
            sl_b = tuple(slice(max(0, d), N - max(0, -d)) for d, N in zip(o, gs))
            diff = E[m][sl_a] - (w[k] if literal else 1.0) * E[m][sl_b]
            bad = np.abs(diff) < tau
            amb[sl_a] |= bad
            amb[sl_b] |= bad
    # a flipped sign changes gE at both ends of the pair; gV then changes over the
    # windows' footprints (the clamped range also covers the reflected samples)
    vox = np.zeros(shape, bool)
    for g in np.argwhere(amb):
        lo = np.maximum(g * s - n // 2, 0)
        hi = np.minimum(g * s + n // 2 - 1, np.array(shape) - 1)
        vox[lo[0]:hi[0] + 1, lo[1]:hi[1] + 1, lo[2]:hi[2] + 1] = True
    return vox


def check_gradient(gV, ref, amb, tol, max_exempt=0.01):
    """Every voxel off by more than tol must be explained by a near tie, and the voxels so
    exempted must be few (at most max_exempt of the volume).  `amb`, the footprint of every
    near-tie term, is wide (a window's n^3 voxels per term); the exempted voxels are those
    of it that actually miss the tolerance."""
    rel = np.abs(gV - ref) / np.max(np.abs(ref))
    bad = rel > tol
    unexplained = bad & ~amb
    print("  max rel err %.3e over all voxels, %.3e off near-tie footprints; %d voxels above %.0e (%.3f %% of the "
          "volume), near-tie footprints cover %.1f %%" % (rel.max(), rel[~amb].max() if (~amb).any() else 0.0,
                                                          int(bad.sum()), tol, 100 * float(bad.mean()),
                                                          100 * float(amb.mean())), flush=True)
    assert not unexplained.any(), np.argwhere(unexplained)[:8]
    assert float(bad.mean()) <= max_exempt, float(bad.mean())


def voxel_explained_by_tie(V, n, s, window, offsets, weights, literal, voxel, tau):
    """True if some center-surround term that reaches gV at `voxel` has |difference| < tau,
    with the features computed by the oracle at just the grid points involved: every window
    covering the voxel (directly or through the border reflection) and the stencil pairs
    (g, g + o) and (g - o, g) of each such window centre g."""
    shape = V.shape
    gs = orc.grid_shape(shape, s)
    w = orc.default_weights(offsets) if weights is None else np.asarray(weights, np.float64)
    off = np.asarray(offsets) // s
    cover = []
    for a in range(3):
        N, v = shape[a], int(voxel[a])
        images = {v, -1 - v, 2 * N - 1 - v}
        cover.append(sorted({g for g in range(gs[a]) for im in images if g * s - n // 2 <= im <= g * s + n // 2 - 1}))
    centres = np.array([[a, b, c] for a in cover[0] for b in cover[1] for c in cover[2]], np.int64)
    pairs = []
    for g in centres:
        for o in off:
            for a, b in ((g, g + o), (g - o, g)):
                if np.all(a >= 0) and np.all(a < gs) and np.all(b >= 0) and np.all(b < gs):
                    pairs.append((tuple(a), tuple(b), o))
    pts = sorted({p for a, b, _ in pairs for p in (a, b)})
    idx = {p: k for k, p in enumerate(pts)}
    E = orc.features_at(V, n, s, window, np.array(pts, np.int64))
    for a, b, o in pairs:
        k = int(np.flatnonzero(np.all(off == o, axis=1))[0])
        diff = E[idx[a]] - (w[k] if literal else 1.0) * E[idx[b]]
        if np.any(np.abs(diff) < tau):
            return True
    return False
