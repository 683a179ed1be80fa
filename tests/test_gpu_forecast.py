"""GPU posterior-predictive simulation against the FP64 oracle on the same
Philox streams, through the C ABI: states, flags and s_-1 bit-exact (integer
decisions taken in FP64 on both sides), locations to 1e-12 of their scale
(device vs libm sqrt / log / sin / cos), at the paper's forecast size
(500 draws x 120 hours, K = 25) on a sample of draws and in full at small
sizes, plus dead ends, empty inputs and argument errors."""
import numpy as np
import pytest
import torch

from oracle import forecast
from paper_2003_03508_amd import synth

from test_gpu_parity import binding, ctx  # noqa: F401

pytestmark = pytest.mark.gpu


def _draws(K, n, seed):
    rng = np.random.default_rng(seed)
    blocks, starts = [], []
    for d in range(n):
        prm = synth.draw_params(rng, K)
        prm.Sigma[:, 1] = rng.uniform(-0.6, 0.6, K) * np.sqrt(prm.Sigma[:, 0] * prm.Sigma[:, 2])
        blocks.append(prm.packed())
        starts.append(rng.dirichlet(np.ones(K)))
    return np.array(blocks), np.array(starts)


def _gpu(binding, ctx, K, blocks, starts, H, seed):
    f64 = dict(dtype=torch.float64, device="cuda")
    r = ctx.simulate(K, torch.as_tensor(blocks, **f64).contiguous(), torch.as_tensor(starts, **f64).contiguous(),
                     H, seed)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in r.items()}


def _compare(got, blocks, starts, K, H, seed, draws):
    for d in draws:
        step, u0 = forecast.philox_draws(seed, d)
        st, fl, xy, first = forecast.simulate_one(blocks[d], starts[d], K, H, step, u0)
        assert got["first"][d] == first
        assert np.array_equal(got["states"][:, d], st), d
        assert np.array_equal(got["flags"][:, d], fl), d
        g = got["xy"][:, d]
        assert np.array_equal(np.isnan(g), np.isnan(xy))
        ok = ~np.isnan(xy)
        assert np.all(np.abs(g[ok] - xy[ok]) <= 1e-12 * (np.abs(xy[ok]) + 1.0)), d


@pytest.mark.parametrize("K,n,H", [(1, 7, 30), (3, 33, 50), (25, 65, 40), (80, 5, 20)])
def test_simulate_matches_oracle(binding, ctx, K, n, H):
    blocks, starts = _draws(K, n, 10 + K)
    got = _gpu(binding, ctx, K, blocks, starts, H, seed=77)
    _compare(got, blocks, starts, K, H, 77, range(n))


def test_paper_forecast_size(binding, ctx):
    """500 draws x 120 hours at K = 25; a sample of draws against the oracle."""
    K, n, H = 25, 500, 120
    blocks, starts = _draws(K, n, 3)
    got = _gpu(binding, ctx, K, blocks, starts, H, seed=2012)
    _compare(got, blocks, starts, K, H, 2012, [0, 1, 255, 256, 257, 498, 499])
    assert got["states"].min() >= 0 and got["states"].max() < K


def test_dead_ends_and_empty(binding, ctx):
    K = 2
    prm, _ = synth.make(K, 10, 5)
    prm.Gamma = np.array([[0.0, 1.0], [0.0, 0.0]])
    blocks = np.array([prm.packed(), prm.packed()])
    starts = np.array([[1.0, 0.0], [0.0, 0.0]])
    got = _gpu(binding, ctx, K, blocks, starts, 6, seed=1)
    _compare(got, blocks, starts, K, 6, 1, [0, 1])
    assert got["first"][1] == -1 and (got["states"][:, 1] == -1).all()
    got = _gpu(binding, ctx, K, blocks, starts, 0, seed=1)
    assert got["states"].shape == (0, 2)
    z = torch.zeros(64, dtype=torch.float64, device="cuda")
    out = torch.zeros(64, dtype=torch.int32, device="cuda")
    for n, K, H in ((1, 0, 5), (-1, 2, 5), (1, 2, -1)):
        rc = binding._lib.hmm_simulate(ctx._h, n, K, z.data_ptr(), z.data_ptr(), H, 0, None, out.data_ptr(),
                                       out.data_ptr(), z.data_ptr(), out.data_ptr())
        assert rc == binding.HMM_E_INVALID_ARG
