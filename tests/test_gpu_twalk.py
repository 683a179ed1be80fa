"""The GPU t-walk (Christen & Fox 2010) against the CPU oracle, through the C
ABI: every proposal (which point, which kernel, the subset, the proposed
point and its log Hastings factor) from the GPU's own pre-state on the same
Philox streams, the likelihood and prior of the proposal, the accept / reject
decision, the kernel counters and history ring, the one-state posterior, and
checkpoint resume.

Tolerances: proposed points to 1e-12 of their scale (FP64 on both sides,
device vs libm pow / log / sin / cos); log factors to 1e-9; log prior to
1e-10 relative; likelihood to the FP32 path's 1e-6 relative; decisions
identical except within a margin of |ln u - ln A| below the likelihood
tolerance (counted, must be rare)."""
import math

import numpy as np
import pytest
import torch

from oracle import mcmc as omcmc
from oracle import twalk
from paper_2003_03508_amd import ess as E
from paper_2003_03508_amd import mcmc as hm

from test_gpu_mcmc import _k1_exact, _problem, _rw_guess, _start, binding, ctx, dev  # noqa: F401

pytestmark = pytest.mark.gpu


def _make(binding, ctx, K, T, C, seed, data_seed, H=64, tuning=None, spread=1.0):
    prm, obs, box = _problem(K, T, data_seed)
    d = binding.to_device(prm, obs)
    rw = _rw_guess(K, obs, prm, c=0.8)
    ch = binding.Chains(ctx, K, C, d["flag"], d["xy"], box, seed=seed, history=H)
    ch.set_state(dev(_start(K, prm, C, spread * rw, np.random.default_rng(0))), dev(rw))
    ch.set_companion(dev(_start(K, prm, C, spread * rw, np.random.default_rng(1))))
    if tuning is not None:
        ch.set_twalk(tuning)
    return ch, prm, obs, box, d


def _compare_twalk(binding, ch, K, obs, box, seed, n_iter, tuning=twalk.DEFAULT):
    """n_iter single t-walk iterations, each checked against the oracle from
    the GPU's pre-state.  Returns (decisions compared, near ties, kernels seen)."""
    C, D = ch.C, ch.D
    f = twalk.hmm_logpost(K, obs.flag, obs.xy, box)
    compared = ties = 0
    kinds = np.zeros(4, dtype=int)
    st, tw = ch.state(), ch.twalk_state()
    x, x2 = st["theta"].cpu().numpy(), tw["theta2"].cpu().numpy()
    for _ in range(n_iter):
        it = st["iterations"]
        ch.step(1, proposal=binding.MCMC_TWALK)
        new, tw_new, pr = ch.state(), ch.twalk_state(), ch.proposal()
        yg = pr["theta"].cpu().numpy()
        code = tw_new["code"].cpu().numpy()
        xn, x2n = new["theta"].cpu().numpy(), tw_new["theta2"].cpu().numpy()
        for c in range(C):
            dr = twalk.philox_draws(seed, it, c, D)
            move_x = dr.uh < 0.5
            h, b = (x[c], x2[c]) if move_x else (x2[c], x[c])
            kind, y, lf, moved = twalk.propose(h, b, dr, tuning)
            assert (code[c] & 1, (code[c] >> 1) & 1, code[c] >> 2) == (int(moved), int(move_x), kind), (it, c)
            scale = np.abs(h) + np.abs(b) + 1.0
            assert np.all(np.abs(yg[c] - y) <= 1e-12 * scale), (it, c, kind)
            keep_x, keep_x2 = x[c], x2[c]
            if not moved:
                assert np.array_equal(xn[c], keep_x) and np.array_equal(x2n[c], keep_x2)
                continue
            kinds[kind] += 1
            lfg = float(pr["logq_fwd"][c])
            if math.isinf(lf):
                assert lfg == lf
            else:
                assert abs(lfg - lf) <= 1e-9 * max(1.0, abs(lf)), (it, c, kind, lfg, lf)
            lp_y = omcmc.log_prior(K, y, box)
            lpg = float(pr["logprior"][c])
            if math.isinf(lp_y):
                assert lpg == lp_y
                ll_y = None
            else:
                assert abs(lpg - lp_y) <= 1e-10 * max(abs(lp_y), 1.0)
                ll_y = omcmc.loglik(K, y, obs.flag, obs.xy)
                assert abs(float(pr["loglik"][c]) - ll_y) <= 1e-6 * max(abs(ll_y), 1.0), (it, c)
            lh = f(h)
            la = (ll_y + lp_y if ll_y is not None else -math.inf) - lh + lf
            lu = math.log(dr.u_acc)
            moved_pt = xn[c] if move_x else x2n[c]
            other_pt, other_old = (x2n[c], keep_x2) if move_x else (xn[c], keep_x)
            assert np.array_equal(other_pt, other_old)
            acc_gpu = np.array_equal(moved_pt, yg[c]) and not np.array_equal(yg[c], h)
            if abs(la - lu) <= 2e-6 * max(abs(lh), 1.0):
                ties += 1
                continue
            compared += 1
            assert acc_gpu == (lu < la), (it, c, kind, la, lu)
            assert np.array_equal(moved_pt, yg[c] if acc_gpu else h)
        x, x2, st = xn, x2n, new
    return compared, ties, kinds


@pytest.mark.parametrize("name,tuning", [("default", twalk.DEFAULT),
                                         ("blow+hop", (0.0, 0.0, 0.5, 6.0, 1.5, 4.0)),
                                         ("traverse+walk", (0.5, 0.5, 0.0, 6.0, 1.5, 4.0))])
def test_twalk_decisions_match_oracle(binding, ctx, name, tuning):
    K, T, C, seed = 3, 3000, 6, 29
    ch, prm, obs, box, _ = _make(binding, ctx, K, T, C, seed, 40, tuning=tuning)
    n_iter = 25
    compared, ties, kinds = _compare_twalk(binding, ch, K, obs, box, seed, n_iter, tuning)
    assert ties <= 2 and compared >= kinds.sum() - 2
    if name == "default":
        assert kinds[0] > 10 and kinds[1] > 10
    elif name == "blow+hop":
        assert kinds[2] > 10 and kinds[3] > 10
    acc = ch.state()["accepts"].cpu().numpy()
    assert 0 < acc.sum() < n_iter * C
    ch.close()


def test_twalk_counters_and_history(binding, ctx):
    K, T, C, H = 2, 1500, 5, 16
    ch, prm, obs, box, _ = _make(binding, ctx, K, T, C, 7, 41, H=H)
    kept = []
    for _ in range(40):
        ch.step(1, proposal=binding.MCMC_TWALK)
        s = ch.state()
        kept.append((s["theta"].cpu().numpy(), (s["loglik"] + s["logprior"]).cpu().numpy()))
    tw, st = ch.twalk_state(), ch.state()
    counts = tw["counts"].cpu().numpy()
    assert np.array_equal(counts[:, :, 1].sum(1), st["accepts"].cpu().numpy())
    assert np.all(counts[:, :, 1] <= counts[:, :, 0]) and counts[:, :, 0].sum() <= 40 * C
    assert counts[:, :, 0].sum() > 30 * C          # empty subsets are rare at D = 16
    hist, hlp, iters = ch.history()
    hist, hlp = hist.cpu().numpy(), hlp.cpu().numpy()
    for it in range(40 - H, 40):
        th, lpost = kept[it]
        assert np.array_equal(hist[it % H], th.astype(np.float32))
        assert np.array_equal(hlp[it % H], lpost)
    # both points' stored likelihoods and priors belong to them
    x2 = tw["theta2"].cpu().numpy()
    for c in range(C):
        ll2 = omcmc.loglik(K, x2[c], obs.flag, obs.xy)
        assert abs(float(tw["loglik2"][c]) - ll2) <= 1e-6 * abs(ll2)
        assert abs(float(tw["logprior2"][c]) - omcmc.log_prior(K, x2[c], box)) <= 1e-9
    ch.close()


def test_twalk_argument_errors(binding, ctx):
    K, T, C = 2, 100, 3
    prm, obs, box = _problem(K, T, 42)
    d = binding.to_device(prm, obs)
    ch = binding.Chains(ctx, K, C, d["flag"], d["xy"], box, seed=1, history=8)
    th = np.tile(hm.theta_from_params(prm.Gamma, prm.p, prm.mu, prm.Sigma), (C, 1))
    with pytest.raises(binding.HMMError):
        ch.set_companion(dev(th))                       # before set_state
    ch.set_state(dev(th), dev(np.full(th.shape[1], 0.01)))
    with pytest.raises(binding.HMMError):
        ch.step(1, proposal=binding.MCMC_TWALK)         # before set_companion
    for bad in ((0.6, 0.6, 0.0, 6, 1.5, 4), (-0.1, 0.5, 0.1, 6, 1.5, 4), (0.5, 0.5, 0, 1.0, 1.5, 4),
                (0.5, 0.5, 0, 6, 0.0, 4), (0.5, 0.5, 0, 6, 1.5, 0.0), (0.5, 0.5, 0, float("nan"), 1.5, 4)):
        with pytest.raises(binding.HMMError):
            ch.set_twalk(bad)
    ch.set_companion(dev(th + 0.01))
    ch.step(3, proposal=binding.MCMC_TWALK)
    assert ch.state()["iterations"] == 3
    ch.close()


def test_twalk_k1_posterior_means(binding, ctx):
    K, T, C, n_burn, n_keep = 1, 60, 64, 800, 2500
    prm, obs, box = _problem(K, T, 5)
    d = binding.to_device(prm, obs)
    ch = binding.Chains(ctx, K, C, d["flag"], d["xy"], box, seed=71, history=n_keep)
    th = hm.theta_from_params(prm.Gamma, prm.p, prm.mu, prm.Sigma)
    rng = np.random.default_rng(3)
    spread = np.array([0.1, 2.0, 2.0, 0.2, 0.2])
    ch.set_state(dev(th + spread * rng.standard_normal((C, 5))), dev(np.full(5, 0.1)))
    ch.set_companion(dev(th + spread * rng.standard_normal((C, 5))))
    ch.step(n_burn, proposal=binding.MCMC_TWALK)
    ch.step(n_keep, proposal=binding.MCMC_TWALK)
    hist, _, iters = ch.history()
    hist = hist.cpu().numpy()
    order = [(iters - n_keep + i) % n_keep for i in range(n_keep)]
    draws = hist[order].astype(np.float64).transpose(1, 0, 2)
    acc = ch.state()["accepts"].cpu().numpy().sum() / (C * (n_burn + n_keep))
    assert 0.1 < acc < 0.8
    Ep, Emx, Ew = _k1_exact(obs)
    p = 1 / (1 + np.exp(-draws[:, :, 0]))
    for est, want in ((p, Ep), (draws[:, :, 1], Emx), (draws[:, :, 3], Ew)):
        assert abs(est.mean() - want) < 4 * E.mcse_mean(est), (est.mean(), want, E.mcse_mean(est))
    ch.close()


def test_twalk_checkpoint_resume_is_bit_identical(binding, ctx):
    K, T, C, H = 3, 2000, 4, 32
    ch, prm, obs, box, d = _make(binding, ctx, K, T, C, 13, 43, H=H, tuning=(0.45, 0.45, 0.05, 5.0, 1.2, 3.0))
    ch.step(9, proposal=binding.MCMC_TWALK)
    image = ch.checkpoint()

    def carry_on(c):
        c.step(11, proposal=binding.MCMC_TWALK)
        c.step(3, proposal=binding.MCMC_RANDOM_WALK)
        c.step(4, proposal=binding.MCMC_TWALK)
        st, tw = c.state(), c.twalk_state()
        hist, hlp, it = c.history()
        return [st["theta"], st["loglik"], st["logprior"], st["accepts"], tw["theta2"], tw["loglik2"],
                tw["logprior2"], tw["counts"], hist, hlp], it

    a, ia = carry_on(ch)
    other = binding.Chains(ctx, K, C, d["flag"], d["xy"], (0.0, 1.0, 0.0, 1.0), seed=5, history=H)
    other.restore(image)
    b, ib = carry_on(other)
    assert ia == ib
    for u, v in zip(a, b):
        assert torch.equal(u, v)
    ch.close()
    other.close()
