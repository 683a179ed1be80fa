"""hmm_validate_params, the host-side parameter check of the C ABI (pure host
code, so it runs without a GPU): a valid set passes; every way of breaking
one block is reported with that block's code, checked in the documented
order; the row-sum tolerance defaults to 1e-12 K."""
import numpy as np
import pytest

from paper_2003_03508_amd import binding, synth


def _prm(K=4, seed=0):
    prm, _ = synth.make(K, 10, seed)
    return [prm.delta.copy(), prm.Gamma.copy(), prm.p.copy(), prm.mu.copy(), prm.Sigma.copy()]


def test_valid_sets_pass():
    for K in (1, 3, 25, 80):
        assert binding.validate_params(*_prm(K, K)) is None
    d, G, p, mu, S = _prm()
    p[:] = [0.0, 1.0, 0.5, 0.25]     # the closed interval
    S[:, 1] = 0.99 * np.sqrt(S[:, 0] * S[:, 2])   # strongly correlated, still SPD
    assert binding.validate_params(d, G, p, mu, S) is None


@pytest.mark.parametrize("block,index,value,code", [
    (0, 1, -1e-3, "delta"), (0, 0, np.nan, "delta"), (0, 2, 0.9, "delta"),
    (1, 5, -1e-9, "Gamma"), (1, 6, np.inf, "Gamma"), (1, 0, 2.0, "Gamma"),
    (2, 3, 1.0 + 1e-12, "p"), (2, 0, -0.1, "p"), (2, 1, np.nan, "p"),
    (3, 7, np.nan, "mu"), (3, 0, -np.inf, "mu"),
    (4, 0, 0.0, "Sigma"), (4, 2, -1.0, "Sigma"), (4, 1, 1e9, "Sigma"), (4, 4, np.nan, "Sigma")])
def test_each_broken_block_is_named(block, index, value, code):
    a = _prm()
    a[block].reshape(-1)[index] = value
    assert binding.validate_params(*a) == code


def test_first_failing_block_in_order_and_tolerance():
    d, G, p, mu, S = _prm()
    p[0] = 2.0
    S[0, 0] = -1.0
    assert binding.validate_params(d, G, p, mu, S) == "p"
    d, G, p, mu, S = _prm()
    G[2, 1] += 1e-9   # row sum off by 1e-9: above the default 4e-12, below 1e-8
    assert binding.validate_params(d, G, p, mu, S) == "Gamma"
    assert binding.validate_params(d, G, p, mu, S, tol=1e-8) is None
    G[2, 1] -= 1e-9 - 2e-12
    assert binding.validate_params(d, G, p, mu, S) is None


def test_bad_shapes_and_arguments():
    d, G, p, mu, S = _prm()
    with pytest.raises(ValueError):
        binding.validate_params(d, G[:2], p, mu, S)
    import ctypes
    what = ctypes.c_int32(7)
    rc = binding._lib.hmm_validate_params(0, None, None, None, None, None, 0.0, ctypes.byref(what))
    assert rc == binding.HMM_E_INVALID_ARG and what.value == 0
