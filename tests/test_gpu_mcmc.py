"""The GPU sampler (Philox streams, parameter transform and prior, MH step,
proposal network and its training) against the CPU oracle, through the C ABI.

Tolerances: Philox uniforms bit-exact (integer arithmetic); normals to
1e-13 (device vs libm log / sin / cos); transform to 1e-13 relative; log
prior to 1e-12 relative (summation order); likelihoods to the FP32 path's
1e-6 relative; accept / reject decisions identical except within a margin
of |ln u - ln A| below the likelihood tolerance (counted, must be rare);
network outputs and gradients (FP32) to 1e-4 of their scale.
"""
import math

import numpy as np
import pytest
import torch

import oracle
from oracle import mcmc as omcmc
from oracle import mlp as omlp
from oracle import philox
from paper_2003_03508_amd import ess as E
from paper_2003_03508_amd import mcmc as hm
from paper_2003_03508_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def binding():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2003_03508_amd import binding as b
    return b


@pytest.fixture(scope="module")
def ctx(binding):
    c = binding.Context(0)
    yield c
    c.close()


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda").contiguous()


# --------------------------------------------------------------------------- Philox
@pytest.mark.parametrize("seed,purpose,it,chain", [(0, 1, 0, 0), (2 ** 64 - 1, 3, 77, 5),
                                                   (123456789012345, 5, 2 ** 32 - 1, 65535)])
def test_philox_uniforms_bit_exact(binding, ctx, seed, purpose, it, chain):
    n = 1000
    got = ctx.philox(seed, purpose, it, chain, n).cpu().numpy()
    want = np.array([philox.uniform2(seed, purpose, it, chain, i) for i in range(n)]).ravel()
    assert np.array_equal(got, want)


def test_philox_normals(binding, ctx):
    n = 4097
    got = ctx.philox(99, 1, 3, 7, n, normal=True).cpu().numpy()
    want = np.array([philox.normal2(99, 1, 3, 7, i) for i in range(n)]).ravel()
    assert np.allclose(got, want, rtol=0, atol=1e-13)


def test_philox_empty(binding, ctx):
    assert ctx.philox(1, 1, 1, 1, 0).numel() == 0


# --------------------------------------------------------------------------- transform and prior
@pytest.mark.parametrize("K", [1, 3, 20, 33, 80])
def test_theta_to_params_and_prior(binding, ctx, K):
    rng = np.random.default_rng(K)
    box = (-3.0, 205.0, 1.0, 199.0)
    n = 5
    th = []
    for i in range(n):
        t = np.concatenate([rng.normal(0, 2, K * (K - 1)), rng.normal(0, 3, K),
                            np.column_stack([rng.uniform(box[0], box[1], K),
                                             rng.uniform(box[2], box[3], K)]).ravel(),
                            rng.normal(5, 2, 2 * K)])
        th.append(t)
    th[-1][K * (K - 1) + K] = box[1] + 0.01          # outside the box
    th = np.stack(th)
    params, lp = ctx.theta_to_params(K, dev(th), box)
    torch.cuda.synchronize()
    params, lp = params.cpu().numpy(), lp.cpu().numpy()
    for i in range(n):
        d, G, p, mu, S = omcmc.to_params(K, th[i])
        want = np.concatenate([d, G.ravel(), p, mu.ravel(), S.ravel()])
        assert np.allclose(params[i], want, rtol=1e-13, atol=1e-300), i
        w = omcmc.log_prior(K, th[i], box)
        if math.isinf(w):
            assert lp[i] == w
        else:
            assert abs(lp[i] - w) <= 1e-12 * max(abs(w), 1.0), (i, lp[i], w)


# --------------------------------------------------------------------------- MH step
def _problem(K, T, seed):
    prm, obs = synth.make(K, T, seed)
    return prm, obs, hm.box_of(obs.flag, obs.xy)


def _rw_guess(K, obs, prm, c=0.5):
    """A rough per-coordinate step (posterior standard deviations from counts)."""
    f = obs.flag.astype(bool)
    T = obs.flag.shape[0]
    nk = T / K
    sl = hm.block_slices(K)
    rw = np.empty(hm.dim(K))
    rw[sl["gamma"]] = 1.0 / math.sqrt(max(nk * 0.02, 1.0))
    rw[sl["p"]] = 1.0 / np.sqrt(nk * prm.p * (1 - prm.p))
    sd = np.sqrt(prm.Sigma[:, [0, 2]])
    rw[sl["mu"]] = (sd / np.sqrt(nk * prm.p)[:, None]).ravel()
    rw[sl["logsigma"]] = np.repeat(np.sqrt(2.0 / (nk * prm.p)), 2)
    return c * rw


def _start(K, prm, C, rw, rng):
    th = hm.theta_from_params(prm.Gamma, prm.p, prm.mu, prm.Sigma)
    return np.stack([th + 0.3 * rw * rng.standard_normal(th.shape[0]) for _ in range(C)])


def _oracle_state(K, th, obs, box):
    return omcmc.loglik(K, th, obs.flag, obs.xy), omcmc.log_prior(K, th, box)


def _compare_steps(binding, ch, K, obs, box, seed, rw, n_iter, net=None, eps=None, theta_tol=1e-12,
                   lq_tol=0.0):
    """Run n_iter single iterations, checking each against the oracle step from
    the GPU's own pre-state.  Returns (decisions compared, near ties)."""
    C = ch.C
    proposal = binding.MCMC_LEARNED if net is not None else binding.MCMC_RANDOM_WALK
    compared = ties = 0
    st = ch.state()
    theta = st["theta"].cpu().numpy()
    for it in range(n_iter):
        it_abs = st["iterations"]
        ch.step(1, proposal=proposal, eps=eps if eps is not None else 0.1)
        new = ch.state()
        pr = ch.proposal()
        th_new = new["theta"].cpu().numpy()
        th_prop = pr["theta"].cpu().numpy()
        for c in range(C):
            ll, lp = _oracle_state(K, theta[c], obs, box)
            r = omcmc.mh_step(K, theta[c], ll, lp, seed, it_abs, c, rw, obs.flag, obs.xy, box, net=net, eps=eps)
            scale = np.abs(theta[c]) + 1.0
            assert np.all(np.abs(th_prop[c] - r["prop"]) <= theta_tol * scale), (it, c)
            lpg = float(pr["logprior"][c])
            if math.isinf(r["lp"]):
                assert lpg == r["lp"]
                continue
            assert abs(lpg - r["lp"]) <= 1e-10 * max(abs(r["lp"]), 1.0) + lq_tol
            llg = float(pr["loglik"][c])
            assert abs(llg - r["ll"]) <= 1e-6 * max(abs(r["ll"]), 1.0), (it, c, llg, r["ll"])
            if net is not None:
                assert abs(float(pr["logq_fwd"][c]) - r["lq_fwd"]) <= lq_tol, (it, c)
            acc_gpu = bool(np.array_equal(th_new[c], th_prop[c])) and not np.array_equal(th_prop[c], theta[c])
            margin = 2e-6 * max(abs(ll), abs(r["ll"]), 1.0) + 3 * lq_tol
            if abs(r["log_ratio"] - r["log_u"]) <= margin:
                ties += 1
            else:
                compared += 1
                assert acc_gpu == r["accept"], (it, c, r["log_ratio"], r["log_u"])
                want = r["prop"] if r["accept"] else theta[c]
                assert np.allclose(th_new[c], want, rtol=0, atol=theta_tol * 10 * scale.max())
        theta = th_new
        st = new
    return compared, ties


def test_random_walk_decisions_match_oracle(binding, ctx):
    K, T, C, seed = 3, 3000, 6, 17
    prm, obs, box = _problem(K, T, 40)
    d = binding.to_device(prm, obs)
    rw = _rw_guess(K, obs, prm, c=0.8)
    ch = binding.Chains(ctx, K, C, d["flag"], d["xy"], box, seed=seed, history=64)
    ch.set_state(dev(_start(K, prm, C, rw, np.random.default_rng(0))), dev(rw))
    compared, ties = _compare_steps(binding, ch, K, obs, box, seed, rw, 25)
    acc = ch.state()["accepts"].cpu().numpy()
    assert acc.sum() > 5 and acc.sum() < 25 * C        # some moves of each kind
    assert ties <= 2 and compared >= 25 * C - 2
    ch.close()


def test_state_after_set_state_and_history_ring(binding, ctx):
    K, T, C, H = 4, 1500, 5, 8
    prm, obs, box = _problem(K, T, 41)
    d = binding.to_device(prm, obs)
    rw = _rw_guess(K, obs, prm)
    ch = binding.Chains(ctx, K, C, d["flag"], d["xy"], box, seed=3, history=H)
    th0 = _start(K, prm, C, rw, np.random.default_rng(1))
    ch.set_state(dev(th0), dev(rw))
    st = ch.state()
    for c in range(C):
        ll, lp = _oracle_state(K, th0[c], obs, box)
        assert abs(float(st["loglik"][c]) - ll) <= 1e-6 * abs(ll)
        assert abs(float(st["logprior"][c]) - lp) <= 1e-10 * max(abs(lp), 1)
    kept = []
    for it in range(20):
        ch.step(1)
        s = ch.state()
        kept.append((s["theta"].cpu().numpy(), (s["loglik"] + s["logprior"]).cpu().numpy()))
    hist, hlp, iters = ch.history()
    assert iters == 20
    hist, hlp = hist.cpu().numpy(), hlp.cpu().numpy()
    for it in range(20 - H, 20):
        th, lpost = kept[it]
        assert np.array_equal(hist[it % H], th.astype(np.float32))
        assert np.array_equal(hlp[it % H], lpost)
    ch.close()


def test_invalid_arguments(binding, ctx):
    K, T = 2, 100
    prm, obs, box = _problem(K, T, 42)
    d = binding.to_device(prm, obs)
    with pytest.raises(binding.HMMError):
        binding.Chains(ctx, 81, 2, d["flag"], d["xy"], box)
    with pytest.raises(binding.HMMError):
        binding.Chains(ctx, K, 2, d["flag"], d["xy"], (1.0, 0.0, 0.0, 1.0))
    ch = binding.Chains(ctx, K, 2, d["flag"], d["xy"], box, history=4)
    with pytest.raises(binding.HMMError):       # untrained network
        ch.step(1, proposal=binding.MCMC_LEARNED)
    with pytest.raises(binding.HMMError):       # not enough history to train
        ch.train(1, lag=1)
    ch.close()


# --------------------------------------------------------------------------- network
def _net_inputs(rng, ch, D):
    H = 256
    P = omlp.count(D, H)
    w = rng.normal(0, 1.0, P)
    # scale each layer like its fan-in so activations stay in tanh's range
    off = 0
    for shp in omlp.sizes(D, H):
        n = int(np.prod(shp))
        w[off:off + n] *= 1.0 / math.sqrt(shp[0]) if len(shp) == 2 else 0.1
        off += n
    return w.astype(np.float32)


@pytest.mark.parametrize("K,B", [(3, 37), (20, 256), (3, 5), (20, 16)])
def test_network_forward_and_gradient(binding, ctx, K, B):
    prm, obs, box = _problem(K, 200, 43)
    d = binding.to_device(prm, obs)
    ch = binding.Chains(ctx, K, 2, d["flag"], d["xy"], box, history=4)
    D = ch.D
    rng = np.random.default_rng(K)
    w = _net_inputs(rng, ch, D)
    ones = np.ones(D)
    ch.set_network(dev(w, torch.float32), dev(np.zeros(D)), dev(ones), dev(ones), lag=1)
    net = ch.network()
    assert net["hidden"] == 256 and net["weights"].numel() == omlp.count(D, 256)
    assert np.array_equal(net["weights"].cpu().numpy(), w)
    X = rng.normal(size=(B, D)).astype(np.float32)
    R = rng.normal(size=(B, D)).astype(np.float32)
    w64 = w.astype(np.float64)
    O = ch.mlp_forward(dev(X, torch.float32)).cpu().numpy()
    Ow, _ = omlp.forward(w64, X.astype(np.float64), D, 256)
    assert np.allclose(O, Ow, rtol=1e-4, atol=1e-4 * np.abs(Ow).max())
    rows, g = ch.mlp_loss_grad(dev(X, torch.float32), dev(R, torch.float32))
    rows, g = rows.cpu().numpy(), g.cpu().numpy()
    rw_ = omlp.loss_rows(w64, X.astype(np.float64), R.astype(np.float64), D, 256)
    assert np.allclose(rows, rw_, rtol=1e-4, atol=1e-5 * np.abs(rw_).max())
    gw = omlp.grad(w64, X.astype(np.float64), R.astype(np.float64), D, 256)
    # per layer, relative to the layer's largest gradient entry
    off = 0
    for shp in omlp.sizes(D, 256):
        n = int(np.prod(shp))
        a, b = g[off:off + n], gw[off:off + n]
        assert np.allclose(a, b, rtol=1e-3, atol=1e-4 * np.abs(b).max()), shp
        off += n
    ch.close()


def _fill_history(binding, ctx, K, T, C, seed, n_iter, H, c_rw=0.8, data_seed=44):
    prm, obs, box = _problem(K, T, data_seed)
    d = binding.to_device(prm, obs)
    rw = _rw_guess(K, obs, prm, c=c_rw)
    ch = binding.Chains(ctx, K, C, d["flag"], d["xy"], box, seed=seed, history=H)
    ch.set_state(dev(_start(K, prm, C, rw, np.random.default_rng(seed))), dev(rw))
    ch.step(n_iter)
    return ch, prm, obs, box, rw, d


def _history_np(ch):
    hist, hlp, iters = ch.history()
    return hist.cpu().numpy(), iters


@pytest.mark.parametrize("back", [0, 10])
def test_standardisation_from_history(binding, ctx, back):
    """First training call: center / in_scale / out_scale from the window
    (the 30 iterations before the current one, or before iteration
    current - back)."""
    K, C, H, lag = 3, 4, 64, 3
    ch, prm, obs, box, rw, _ = _fill_history(binding, ctx, K, 1500, C, 9, 50, H)
    hist, iters = _history_np(ch)
    ch.train(1, batch=8, lag=lag, lr=1e-3, window=30, window_end=iters - back if back else 0)
    net = ch.network()
    t1 = iters - back
    t0 = t1 - 30
    win = np.stack([hist[t % H] for t in range(t0, t1)]).astype(np.float64)     # (n, C, D)
    moves = np.stack([hist[(t + lag) % H] - hist[t % H] for t in range(t0, t1 - lag)]).astype(np.float64)
    fl = 0.1 * rw
    center = win.reshape(-1, ch.D).mean(axis=0)
    ins = np.maximum(win.reshape(-1, ch.D).std(axis=0, ddof=1), fl)
    outs = np.maximum(moves.reshape(-1, ch.D).std(axis=0, ddof=1), fl)
    assert np.allclose(net["center"].cpu().numpy(), center, rtol=1e-12, atol=1e-12)
    assert np.allclose(net["in_scale"].cpu().numpy(), ins, rtol=1e-9)
    assert np.allclose(net["out_scale"].cpu().numpy(), outs, rtol=1e-9)
    assert net["lag"] == lag and net["trained"]
    # the least-squares start of the linear part (one Adam step moves each
    # weight by at most ~lr = 1e-3)
    D = ch.D
    X = ((np.stack([hist[t % H] for t in range(t0, t1 - lag)]).astype(np.float64) - center) / ins).reshape(-1, D)
    Rm = (moves / outs).reshape(-1, D)
    w = net["weights"].cpu().numpy().astype(np.float64)
    P = omlp.count(D, 256)
    a_got, b_got, ls_got = w[P - D:], w[P - 3 * D:P - 2 * D], w[P - 2 * D:P - D]
    for j in range(D):
        A = np.column_stack([X[:, j], np.ones(X.shape[0])])
        (a, b), res, *_ = np.linalg.lstsq(A, Rm[:, j], rcond=None)
        s2 = np.sum((Rm[:, j] - a * X[:, j] - b) ** 2) / (X.shape[0] - 2)
        assert abs(a_got[j] - a) <= 2e-3 + 1e-4 * abs(a), (j, a_got[j], a)
        assert abs(b_got[j] - b) <= 2e-3 + 1e-4 * abs(b), (j, b_got[j], b)
        assert abs(ls_got[j] - 0.5 * math.log(s2)) <= 2e-3, (j, ls_got[j], 0.5 * math.log(s2))
    with pytest.raises(binding.HMMError):       # the lag is fixed by the first call
        ch.train(1, batch=8, lag=lag + 1)
    with pytest.raises(binding.HMMError):       # the window must end at or before now
        ch.train(1, batch=8, lag=lag, window_end=iters + 1)
    # a reset forgets the network and the standardisation
    ch.reset_proposal(seed=4)
    net = ch.network()
    assert not net["trained"]
    w = net["weights"].cpu().numpy()
    D = ch.D
    tail = w[omlp.count(D, 256) - (256 * 2 * D + 2 * D + D):]
    assert np.all(tail == 0)                        # W3, b3 and the skip are zero
    assert np.any(w[:D * 256] != 0)                 # W1 re-initialised
    ch.train(2, batch=8, lag=lag + 1, lr=1e-3)      # a new lag is allowed
    assert ch.network()["lag"] == lag + 1
    with pytest.raises(binding.HMMError):
        ch.step(1, proposal=binding.MCMC_LEARNED, eps=1.0)   # eps must lie in (0, 1)
    ch.close()


def test_training_step_matches_oracle(binding, ctx):
    """One Adam step: minibatch drawn from the history with Philox, gradient
    by backpropagation, update -- against the FP64 oracle on the same pairs."""
    K, C, H, lag, B, lr, seed = 3, 5, 64, 2, 48, 1e-3, 12
    ch, prm, obs, box, rw, _ = _fill_history(binding, ctx, K, 1500, C, seed, 50, H)
    D = ch.D
    rng = np.random.default_rng(7)
    w0 = _net_inputs(rng, ch, D)
    center = rng.normal(0, 0.1, D) + ch.state()["theta"].cpu().numpy().mean(axis=0)
    ins = np.exp(rng.normal(0, 0.3, D)) * rw * 3
    outs = np.exp(rng.normal(0, 0.3, D)) * rw
    ch.set_network(dev(w0, torch.float32), dev(center), dev(ins), dev(outs), lag=lag)
    hist, iters = _history_np(ch)
    losses = ch.train(1, batch=B, lag=lag, lr=lr, window=0)["loss"].cpu().numpy()
    w1 = ch.network()["weights"].cpu().numpy().astype(np.float64)
    # the oracle's minibatch: time and chain from Philox purpose 4, step 0
    t1, t0 = iters, iters - min(H, iters)
    span = t1 - lag - t0
    X = np.empty((B, D), dtype=np.float32)
    R = np.empty((B, D), dtype=np.float32)
    for b in range(B):
        u0, u1 = philox.uniform2(seed, philox.MINIBATCH, 0, 0, b)
        t = t0 + min(span - 1, int(u0 * span))
        c = min(C - 1, int(u1 * C))
        x = hist[t % H, c].astype(np.float64)
        y = hist[(t + lag) % H, c].astype(np.float64)
        X[b] = (x - center) / ins
        R[b] = (y - x) / outs
    w0d = w0.astype(np.float64)
    g = omlp.grad(w0d, X.astype(np.float64), R.astype(np.float64), D, 256)
    assert abs(losses[0] - omlp.loss(w0d, X.astype(np.float64), R.astype(np.float64), D, 256)) <= \
        1e-4 * abs(losses[0])
    # Adam's first step: m_hat = g, v_hat = g^2 -> w1 = w0 - lr g / (|g| + 1e-8)
    want = w0d - lr * g / (np.abs(g) + 1e-8)
    off = 0
    for shp in omlp.sizes(D, 256):
        n = int(np.prod(shp))
        gl = g[off:off + n]
        big = np.abs(gl) > 1e-3 * np.abs(gl).max()      # the update's sign is decided
        assert big.mean() > 0.5, shp
        assert np.allclose(w1[off:off + n][big], want[off:off + n][big], rtol=0, atol=1e-3 * lr + 1e-7), shp
        off += n
    ch.close()


def test_held_out_selection(binding, ctx):
    """With a held-out part of the window the call keeps the weights of the
    lowest held-out loss; the held-out pairs and losses match the oracle."""
    K, C, H, lag, vb, ve, steps, seed = 3, 4, 128, 2, 64, 5, 20, 14
    ch, prm, obs, box, rw, _ = _fill_history(binding, ctx, K, 1500, C, seed, 100, H)
    D = ch.D
    hist, iters = _history_np(ch)
    r = ch.train(steps, batch=32, lag=lag, lr=3e-3, window=80, holdout=0.25, val_every=ve, val_batch=vb)
    val = r["val"].cpu().numpy()
    assert val.shape[0] == 1 + -(-steps // ve)
    best_i = int(np.argmin(val))
    assert r["best_step"] == (-1 if best_i == 0 else min(best_i * ve, steps) - 1)
    net = ch.network()
    center = net["center"].cpu().numpy()
    ins = net["in_scale"].cpu().numpy()
    outs = net["out_scale"].cpu().numpy()
    # the held-out pairs: starts in [tv, t1 - lag), Philox purpose 6, step word 0
    t1 = iters
    t0 = t1 - 80
    tv = t0 + int(math.floor(0.75 * (t1 - t0)))
    span = t1 - lag - tv
    X = np.empty((vb, D))
    R = np.empty((vb, D))
    for b in range(vb):
        u0, u1 = philox.uniform2(seed, 6, 0, 0, b)
        t = tv + min(span - 1, int(u0 * span))
        c = min(C - 1, int(u1 * C))
        x = hist[t % H, c].astype(np.float64)
        y = hist[(t + lag) % H, c].astype(np.float64)
        X[b] = ((x - center) / ins).astype(np.float32)
        R[b] = ((y - x) / outs).astype(np.float32)
    w = net["weights"].cpu().numpy().astype(np.float64)
    kept = omlp.loss(w, X, R, D, 256)               # mean row loss, as the kernel sums rows / B
    assert abs(kept - val.min()) <= 1e-4 * abs(val.min()) + 1e-3, (kept, val.min())
    ch.close()


def test_learned_decisions_match_oracle(binding, ctx):
    K, T, C, seed = 3, 2000, 6, 8
    ch, prm, obs, box, rw, _ = _fill_history(binding, ctx, K, T, C, seed, 200, 200)
    ch.train(100, batch=128, lag=3, lr=1e-3)
    net = ch.network()
    w = net["weights"].cpu().numpy().astype(np.float64)
    center = net["center"].cpu().numpy()
    ins = net["in_scale"].cpu().numpy()
    outs = net["out_scale"].cpu().numpy()
    D = ch.D

    def move(theta):
        return omlp.move(w, theta, center, ins, outs, D, 256)

    # FP32 network: theta' agrees to ~1e-6 of the step, the log densities to ~1e-4
    compared, ties = _compare_steps(binding, ch, K, obs, box, seed, rw, 15, net=move, eps=0.25,
                                    theta_tol=1e-5, lq_tol=2e-3)
    assert ties <= 3 and compared >= 15 * C - 3
    ch.close()


def test_learned_decisions_match_oracle_k20(binding, ctx):
    """The sampled workload's size: K = 20 (D = 480 parameters), the learned
    mixture (network trained on the chains' own history, eps = 0.1), each
    decision against the oracle's MH step from the GPU's pre-state, with a
    short observation sequence."""
    K, T, C, seed = 20, 3000, 4, 21
    ch, prm, obs, box, rw, _ = _fill_history(binding, ctx, K, T, C, seed, 240, 240, c_rw=0.3, data_seed=45)
    ch.train(150, batch=64, lag=5, lr=1e-3)
    net = ch.network()
    w = net["weights"].cpu().numpy().astype(np.float64)
    center = net["center"].cpu().numpy()
    ins = net["in_scale"].cpu().numpy()
    outs = net["out_scale"].cpu().numpy()
    D = ch.D
    assert D == 480

    def move(theta):
        return omlp.move(w, theta, center, ins, outs, D, 256)

    compared, ties = _compare_steps(binding, ch, K, obs, box, seed, rw, 8, net=move, eps=0.1,
                                    theta_tol=1e-5, lq_tol=2e-2)
    assert ties <= 2 and compared >= 8 * C - 2
    acc = ch.state()["accepts"].cpu().numpy()
    print(f"K=20 learned mixture: {compared} decisions compared, {ties} near ties, accepts {acc.tolist()}")
    ch.close()


# --------------------------------------------------------------------------- posterior checks
def _k1_exact(obs):
    from scipy import integrate
    from scipy.special import digamma
    f = obs.flag.astype(bool)
    n1, n0 = int(f.sum()), int((~f).sum())
    a, b = omcmc.gamma_shape_rate(0, 1)
    logf = lambda q: (n1 + a - 1) * math.log(q) + n0 * math.log1p(-q) - b * q
    grid = np.linspace(1e-6, 1 - 1e-6, 20001)
    vals = np.array([logf(q) for q in grid])
    m, mode = vals.max(), grid[np.argmax(vals)]
    Z = integrate.quad(lambda q: math.exp(logf(q) - m), 0, 1, points=[mode], limit=200)[0]
    Ep = integrate.quad(lambda q: q * math.exp(logf(q) - m), 0, 1, points=[mode], limit=200)[0] / Z
    x = obs.xy.reshape(-1, 2)[f, 0]
    S = float(((x - x.mean()) ** 2).sum())
    return Ep, float(x.mean()), math.log((S + 1) / 2) - digamma((n1 + 1) / 2)


def _k1_draws(binding, ctx, proposal, seed, n_burn=500, n_keep=2000, train=False):
    K, T, C = 1, 60, 64
    prm, obs, box = _problem(K, T, 5)
    d = binding.to_device(prm, obs)
    f = obs.flag.astype(bool)
    n1 = f.sum()
    x = obs.xy.reshape(-1, 2)[f]
    rw = 1.2 * np.array([0.15, x[:, 0].std() / math.sqrt(n1), x[:, 1].std() / math.sqrt(n1),
                         math.sqrt(2 / n1), math.sqrt(2 / n1)])
    ch = binding.Chains(ctx, K, C, d["flag"], d["xy"], box, seed=seed, history=n_keep)
    th = hm.theta_from_params(prm.Gamma, prm.p, prm.mu, prm.Sigma)
    ch.set_state(dev(np.tile(th, (C, 1))), dev(rw))
    ch.step(n_burn)
    if train:
        ch.train(400, batch=256, lag=2, lr=2e-3, window=n_burn)
    ch.step(n_keep, proposal=proposal, eps=0.2)
    hist, _, iters = ch.history()
    hist = hist.cpu().numpy()
    order = [(iters - n_keep + i) % n_keep for i in range(n_keep)]
    draws = hist[order].astype(np.float64).transpose(1, 0, 2)   # (C, n, D)
    acc = ch.state()["accepts"].cpu().numpy()
    ch.close()
    return draws, obs, acc


@pytest.mark.parametrize("learned", [False, True])
def test_k1_posterior_means(binding, ctx, learned):
    prop = binding.MCMC_LEARNED if learned else binding.MCMC_RANDOM_WALK
    draws, obs, acc = _k1_draws(binding, ctx, prop, seed=61 + learned, train=learned)
    Ep, Emx, Ew = _k1_exact(obs)
    p = 1 / (1 + np.exp(-draws[:, :, 0]))
    for est, want in ((p, Ep), (draws[:, :, 1], Emx), (draws[:, :, 3], Ew)):
        assert abs(est.mean() - want) < 4 * E.mcse_mean(est), (est.mean(), want, E.mcse_mean(est))


def test_checkpoint_resume_is_bit_identical(binding, ctx):
    """A sampler restored from a checkpoint continues exactly as the saved
    one: MH steps of both proposals and further training."""
    K, T, C, H = 3, 2000, 4, 64
    ch, prm, obs, box, rw, d = _fill_history(binding, ctx, K, T, C, 21, 30, H)
    ch.train(40, batch=64, lag=2, lr=1e-3)
    ch.step(5, proposal=binding.MCMC_LEARNED, eps=0.2)
    image = ch.checkpoint()

    def carry_on(c):
        c.step(7, proposal=binding.MCMC_LEARNED, eps=0.2)
        c.train(10, batch=64, lag=2, lr=1e-3)
        c.step(6, proposal=binding.MCMC_RANDOM_WALK)
        st = c.state()
        hist, hlp, it = c.history()
        net = c.network()
        return [st["theta"], st["loglik"], st["logprior"], st["accepts"], hist, hlp, net["weights"],
                net["center"], net["in_scale"], net["out_scale"]], (it, st["iterations"], net["lag"])

    a, a_meta = carry_on(ch)
    other = binding.Chains(ctx, K, C, d["flag"], d["xy"], (0.0, 1.0, 0.0, 1.0), seed=999, history=H)
    other.restore(image)
    b, b_meta = carry_on(other)
    assert a_meta == b_meta
    for x, y in zip(a, b):
        assert torch.equal(x, y)
    # images of another shape or damaged ones are refused
    wrong = binding.Chains(ctx, K, C + 1, d["flag"], d["xy"], box, history=H)
    with pytest.raises(binding.HMMError):
        wrong.restore(image)
    with pytest.raises(binding.HMMError):
        other.restore(b"\0" * len(image))
    with pytest.raises(binding.HMMError):
        other.restore(image[:-1])
    for c in (ch, other, wrong):
        c.close()


def test_trained_proposal_beats_random_walk():
    """What the trained network gains: on a K=3 posterior (D=21), after the
    same adapted random-walk burn-in, the learned mixture proposal (lag 10,
    least-squares start + Adam steps kept by held-out loss) gives several
    times the effective samples per iteration of the random walk -- median
    over coordinates, minimum, and the log posterior -- at the same posterior
    means (within Monte Carlo error)."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2003_03508_amd import binding
    ctx = binding.Context(0)
    K, T, C, N, seed = 3, 3000, 16, 1500, 3
    prm, obs, box = _problem(K, T, 53)
    d = binding.to_device(prm, obs)
    D = hm.dim(K)
    H = 2000 + 2 * N
    rw = _rw_guess(K, obs, prm, c=1.0) * 2.38 / math.sqrt(D)
    ch = binding.Chains(ctx, K, C, d["flag"], d["xy"], box, seed=seed, history=H)
    ch.set_state(dev(_start(K, prm, C, rw, np.random.default_rng(0))), dev(rw))

    def window(n):
        hist, hlp, it = ch.history()
        idx = [(it - n + i) % H for i in range(n)]
        return hist[idx].cpu().numpy().transpose(1, 0, 2).astype(np.float64), hlp[idx].cpu().numpy().T

    scale = 1.0
    for _ in range(4):                      # burn-in with scale adaptation
        a0 = int(ch.state()["accepts"].sum())
        ch.step(500)
        acc = (int(ch.state()["accepts"].sum()) - a0) / (500 * C)
        scale *= math.exp(3.0 * (acc - 0.234))
        rw = scale * 2.38 / math.sqrt(D) * window(500)[0][:, 100:].reshape(-1, D).std(axis=0)
        ch.set_rw_scale(dev(rw))
    start = ch.state()["theta"].clone()
    burn_end = ch.state()["iterations"]
    r = ch.train(300, batch=256, lag=10, lr=1e-4, window=1500, window_end=burn_end, holdout=0.2,
                 val_every=25, val_batch=1024)
    out = {}
    for name, prop in (("rw", binding.MCMC_RANDOM_WALK), ("learned", binding.MCMC_LEARNED)):
        ch.set_state(start, dev(rw))
        ch.step(N, proposal=prop, eps=0.1)
        w, lp = window(N)
        e = E.ess_columns(w)
        out[name] = dict(med=np.median(e), min=e.min(), lp=E.ess(lp), mean=w.reshape(-1, D).mean(axis=0),
                         mcse=np.array([E.mcse_mean(w[:, :, j]) for j in range(D)]))
    ch.close()
    ctx.close()
    a, b = out["rw"], out["learned"]
    assert b["med"] >= 2.0 * a["med"], (a["med"], b["med"])
    assert b["lp"] >= 2.0 * a["lp"], (a["lp"], b["lp"])
    assert b["min"] >= a["min"], (a["min"], b["min"])
    z = np.abs(a["mean"] - b["mean"]) / np.sqrt(a["mcse"] ** 2 + b["mcse"] ** 2)
    assert np.all(z < 4.5), z.max()
