"""Sequential LMS / NLMS / RLS weights on the GPU (Sec. 2, fusion paragraph; Fig. 6)
against the FP64 oracle's recursions on the same S_m: weights, samples per pass and the
learning curve (squared a priori errors in update order), with and without re-adaptation
every N sections; the fused map S with those weights; RLS with unit forgetting factor
against the closed-form least-squares weights."""
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


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


# rule, parameters, grid, sections, masked, passes
CASES = [
    ("lms", dict(mu=0.05), (9, 14, 11), 0, True, 3),
    ("nlms", dict(mu=0.5, eps=1e-3), (9, 14, 11), 0, False, 2),
    ("rls", dict(lam=0.99, delta=0.1), (9, 14, 11), 0, True, 1),
    ("nlms", dict(mu=0.3, eps=0.0), (7, 23, 9), 5, True, 2),
    ("rls", dict(lam=1.0, delta=1.0), (7, 23, 9), 4, False, 2),
    ("lms", dict(mu=0.02), (6, 70, 5), 1, False, 1),   # one group per inline section
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_adapt_matches_oracle(torch_sal, case):
    torch, sal = torch_sal
    rule, prm, gs, N, masked, passes = CASES[case]
    print("sequential %s %s grid %s sections %d passes %d" % (rule, prm, gs, N, passes), flush=True)
    rng = np.random.default_rng(700 + case)
    Sm = rng.uniform(0.1, 1.5, size=(3,) + gs).astype(np.float32)
    D = (Sm[0] * 0.6 - 0.3 * Sm[1] + 0.9 * Sm[2] + 0.1 * rng.standard_normal(gs)).astype(np.float32)
    mask = (rng.uniform(size=gs) < 0.6).astype(np.uint8) if masked else None
    w0 = (0.2, 0.1, -0.05)
    cfg = sal.Config(fusion=rule, wfix=w0, sections=N, passes=passes, mu=prm.get("mu", 0.5),
                     eps=prm.get("eps", 1e-6), lam=prm.get("lam", 1.0), delta=prm.get("delta", 0.0))
    cap = int(np.prod(gs)) * passes
    Smd, Dd = _dev(torch, Sm), _dev(torch, D)
    Md = None if mask is None else _dev(torch, mask)
    W, err, cnt = sal.adapt_weights(Smd, cfg, Dd, Md, cap)
    W, err, cnt = W.cpu().numpy(), err.cpu().numpy(), cnt.cpu().numpy()
    Wo, cnto, erro = orc.adapt_sequential(Sm, D, mask, rule, mu=cfg.mu, eps=cfg.eps, lam=cfg.lam,
                                          delta=prm.get("delta", 1.0), w0=w0, passes=passes, sections=N, cap=cap)
    assert np.array_equal(cnt, cnto)
    assert np.all(W[:, 3] == 0)
    rel = np.max(np.abs(W[:, :3] - Wo)) / np.abs(Wo).max()
    print("  weights rel err %.2e over %d groups, %d samples" % (rel, W.shape[0], int(cnt.sum())), flush=True)
    assert rel < 1e-10
    for k in range(W.shape[0]):
        n = int(cnto[k]) * passes
        assert np.max(np.abs(err[k, :n] - erro[k, :n])) <= 1e-6 * max(erro[k, :n].max(), 1e-30)
    # sal_fuse with the same rule: the same weights, and S their combine
    shape = tuple(g * 2 for g in gs)
    S, Wf = sal.fuse(Smd, shape, 2, rule, w0, cfg.delta, Dd, Md, sections=N, mu=cfg.mu, eps=cfg.eps, lam=cfg.lam,
                     passes=passes)
    Wf = Wf.cpu().numpy().reshape(-1, 4)
    assert np.array_equal(Wf, W)
    So = orc.combine_sections(Sm, Wf[:, :3], N, shape, 2) if N else orc.combine(Sm, Wf[0, :3], shape, 2)
    assert np.max(np.abs(S.cpu().numpy() - So)) <= 1e-6 * np.abs(So).max()


def test_rls_unit_forgetting_matches_least_squares(torch_sal):
    """RLS with lambda = 1, P0 = I / delta and W0 = 0 ends at ADAPT_LS with ridge delta."""
    torch, sal = torch_sal
    rng = np.random.default_rng(77)
    gs = (16, 21, 13)
    Sm = _dev(torch, rng.uniform(0.1, 1.5, size=(3,) + gs).astype(np.float32))
    D = _dev(torch, rng.uniform(size=gs).astype(np.float32))
    mask = _dev(torch, (rng.uniform(size=gs) < 0.5).astype(np.uint8))
    cfg = sal.Config(fusion="rls", wfix=(0.0, 0.0, 0.0), lam=1.0, delta=0.25)
    W, _, _ = sal.adapt_weights(Sm, cfg, D, mask)
    _, Wls = sal.fuse(Sm, tuple(2 * g for g in gs), 2, "adapt_ls", delta=0.25, D=D, mask=mask)
    W, Wls = W.cpu().numpy()[0, :3], Wls.cpu().numpy()[:3]
    assert np.max(np.abs(W - Wls)) < 1e-9 * np.abs(Wls).max()


def test_nlms_on_the_survey_section(torch_sal):
    """NLMS over the survey-size grid (128 x 200 x 300) with the fit mask on its middle inline
    section, two passes: weights and learning curve against the oracle."""
    torch, sal = torch_sal
    w = synth.workload("survey")
    gs = synth.grid_shape(w.spec.shape, w.s)
    rng = np.random.default_rng(78)
    Sm = rng.uniform(0.0, 2.0, size=(3,) + gs).astype(np.float32)
    D = (rng.uniform(size=gs) < 0.2).astype(np.float32)
    mask = np.zeros(gs, np.uint8)
    mask[:, gs[1] // 2, :] = 1
    cfg = sal.Config(fusion="nlms", wfix=(1 / 3, 1 / 3, 1 / 3), mu=0.2, eps=1e-6, passes=2)
    cap = 2 * int(mask.sum())
    W, err, cnt = sal.adapt_weights(_dev(torch, Sm), cfg, _dev(torch, D), _dev(torch, mask), cap)
    Wo, cnto, erro = orc.adapt_sequential(Sm, D, mask, "nlms", mu=0.2, eps=1e-6, w0=cfg.wfix, passes=2, cap=cap)
    assert int(cnt.item()) == int(cnto[0]) == int(mask.sum())
    assert np.max(np.abs(W.cpu().numpy()[0, :3] - Wo[0])) < 1e-10 * np.abs(Wo).max()
    e = err.cpu().numpy()[0]
    assert np.max(np.abs(e - erro[0])) <= 1e-6 * erro[0].max()
