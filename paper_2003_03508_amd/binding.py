"""Thin ctypes binding of the C ABI in include/hmm.h.

Argument marshalling only: torch tensors are checked (device, dtype, layout)
and their device pointers and the current HIP stream are handed to the
library; every step of the computation runs in the library's kernels.  If the
compiled library is missing the import fails -- there is no fallback.
"""
import ctypes
import os
import numpy as np

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhmm.so")

HMM_OK = 0
HMM_E_INVALID_ARG = -1
HMM_E_UNSUPPORTED = -2
HMM_E_DEVICE = -3
HMM_E_NOMEM = -4

SERIAL_F32 = 0
BLOCKED_F32 = 1
BLOCKED_BF16 = 2
BLOCKED_F16 = 3
BLOCKED_BF16_SPLIT = 4
BLOCKED_F16_SPLIT = 5
EMIS_POISSON = 1
EMIS_GAUSS1D = 2
ALGOS = {"serial_f32": SERIAL_F32, "blocked_f32": BLOCKED_F32,
         "blocked_bf16": BLOCKED_BF16, "blocked_f16": BLOCKED_F16,
         "blocked_bf16_split": BLOCKED_BF16_SPLIT, "blocked_f16_split": BLOCKED_F16_SPLIT}

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with "
                      "`python -m paper_2003_03508_amd.build` (no CPU fallback exists)")

_lib = ctypes.CDLL(LIB_PATH)
_vp = ctypes.c_void_p
_i32, _i64 = ctypes.c_int32, ctypes.c_int64

_lib.hmm_ctx_create.argtypes = [ctypes.POINTER(_vp), ctypes.c_int]
_lib.hmm_ctx_destroy.argtypes = [_vp]
_lib.hmm_loglik.argtypes = [_vp, _i32, _vp, _vp, _vp, _vp, _vp, _i64, _vp, _vp, _i32, _vp, _vp]
_lib.hmm_loglik_noalloc.argtypes = [_i32, _vp, _vp, _vp, _vp, _vp, _i64, _vp, _vp, _i32, _vp, _vp]
_lib.hmm_emission.argtypes = [_vp, _i32, _vp, _vp, _vp, _i64, _vp, _vp, _vp, _vp, _vp, _vp]
_lib.hmm_ctx_set_blocking.argtypes = [_vp, _i64, _i32]
_lib.hmm_blocked_plan.argtypes = [_vp, _i32, _i64, ctypes.POINTER(_i64), ctypes.POINTER(_i64),
                                  ctypes.POINTER(_i32)]
_lib.hmm_ctx_profile.argtypes = [_vp, _i32]
_lib.hmm_ctx_profile_read.argtypes = [_vp, ctypes.POINTER(_i64), ctypes.POINTER(ctypes.c_double)]
_lib.hmm_loglik_batched.argtypes = [_vp, _i32, _vp, _vp, _vp, _vp, _i64, _vp, _vp, _vp, _i64, _i32, _vp, _vp]
_lib.hmm_ctx_set_batch_graph.argtypes = [_vp, _i32]
_lib.hmm_ctx_set_batch_persistent.argtypes = [_vp, _i32]
_lib.hmm_ctx_set_packing.argtypes = [_vp, _i32]
_lib.hmm_autotune_batched.argtypes = [_vp, _i32, _vp, _vp, _vp, _vp, _i64, _vp, _vp, _vp, _i64, _i32, _vp,
                                      _i32, _vp]
_lib.hmm_loglik_kind.argtypes = [_vp, _i32, _i32, _vp, _vp, _vp, _vp, _i64, _vp, _i32, _vp, _vp]
_lib.hmm_theta_to_params.argtypes = [_vp, _i32, _i32, _vp, _vp, _vp, _vp, _vp]
_lib.hmm_philox.argtypes = [_vp, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, _i64,
                            _i32, _vp, _vp]
_lib.mcmc_create.argtypes = [_vp, _i32, _i32, _i64, _vp, _vp, _vp, ctypes.c_uint64, _i64, ctypes.POINTER(_vp)]
_lib.mcmc_destroy.argtypes = [_vp]
_lib.mcmc_set_state.argtypes = [_vp, _vp, _vp, _vp]
_lib.mcmc_set_rw_scale.argtypes = [_vp, _vp, _vp]
_lib.mcmc_step.argtypes = [_vp, _i32, _i32, ctypes.c_double, _vp]
class TrainOpts(ctypes.Structure):
    """Mirror of mcmc_train_opts in include/hmm.h."""
    _fields_ = [("steps", _i32), ("batch", _i32), ("lag", _i32), ("lr", ctypes.c_double),
                ("weight_decay", ctypes.c_double), ("window", _i64), ("window_end", _i64),
                ("holdout", ctypes.c_double), ("val_every", _i32), ("val_batch", _i32)]


_lib.mcmc_train_proposal.argtypes = [_vp, ctypes.POINTER(TrainOpts), _vp, _vp, _vp, ctypes.POINTER(_i32)]
_lib.mcmc_reset_proposal.argtypes = [_vp, ctypes.c_uint64, _vp]
_lib.mlp_forward.argtypes = [_vp, _i32, _vp, _vp, _vp]
_lib.mlp_loss_grad.argtypes = [_vp, _i32, _vp, _vp, _vp, _vp, _vp]
_lib.mlp_set_weights.argtypes = [_vp, _vp, _vp, _vp, _vp, _i32, _vp]
_lib.mcmc_checkpoint_size.argtypes = [_vp, ctypes.POINTER(_i64)]
_lib.mcmc_checkpoint_save.argtypes = [_vp, _vp, _i64, _vp]
_lib.mcmc_checkpoint_load.argtypes = [_vp, _vp, _i64, _vp]
_lib.mcmc_set_companion.argtypes = [_vp, _vp, _vp]
_lib.hmm_posterior.argtypes = [_vp, _i32, _vp, _vp, _vp, _vp, _vp, _i64, _vp, _vp, _vp, _vp, _vp, _vp]
_lib.hmm_loglik_grad.argtypes = [_vp, _i32, _vp, _vp, _vp, _vp, _vp, _i64, _vp, _vp, _vp, _vp, _vp]
_lib.hmm_validate_params.argtypes = [_i32, _vp, _vp, _vp, _vp, _vp, ctypes.c_double, _vp]
_lib.hmm_em_step.argtypes = [_vp, _i32, _vp, _vp, _vp, _vp, _vp, _i64, _vp, _vp, _vp, _vp, _vp]
_lib.hmm_viterbi.argtypes = [_vp, _i32, _vp, _vp, _vp, _vp, _vp, _i64, _vp, _vp, _vp, _vp, _vp, _vp]
_lib.hmm_simulate.argtypes = [_vp, _i32, _i32, _vp, _vp, _i32, ctypes.c_uint64, _vp, _vp, _vp, _vp, _vp]
_lib.mcmc_set_twalk.argtypes = [_vp, _vp]


class McmcView(ctypes.Structure):
    """Mirror of mcmc_view in include/hmm.h."""
    _fields_ = [("K", _i32), ("n_chains", _i32), ("dim", _i32),
                ("iterations", _i64), ("history_len", _i64),
                ("theta", _vp), ("loglik", _vp), ("logprior", _vp),
                ("theta_prop", _vp), ("loglik_prop", _vp), ("logprior_prop", _vp), ("logq_fwd", _vp),
                ("accepts", _vp), ("history", _vp), ("history_logpost", _vp),
                ("net_weights", _vp), ("net_count", _i64), ("net_hidden", _i32),
                ("center", _vp), ("in_scale", _vp), ("out_scale", _vp),
                ("lag", _i32), ("trained", _i32),
                ("theta2", _vp), ("loglik2", _vp), ("logprior2", _vp), ("twalk_counts", _vp),
                ("twalk_code", _vp), ("companion", _i32)]


_lib.mcmc_view_get.argtypes = [_vp, ctypes.POINTER(McmcView)]
_lib.hmm_status_string.restype = ctypes.c_char_p
_lib.hmm_status_string.argtypes = [ctypes.c_int]
for _f in ("hmm_ctx_create", "hmm_ctx_destroy", "hmm_loglik", "hmm_loglik_noalloc", "hmm_emission",
           "hmm_ctx_set_blocking", "hmm_blocked_plan", "hmm_ctx_profile", "hmm_ctx_profile_read",
           "hmm_loglik_batched", "hmm_ctx_set_batch_graph", "hmm_ctx_set_batch_persistent",
           "hmm_ctx_set_packing", "hmm_autotune_batched",
           "hmm_theta_to_params", "hmm_philox", "hmm_loglik_kind", "mcmc_create", "mcmc_destroy", "mcmc_set_state",
           "mcmc_set_rw_scale", "mcmc_step", "mcmc_train_proposal", "mcmc_reset_proposal", "mcmc_view_get",
           "mlp_forward",
           "mlp_loss_grad", "mlp_set_weights", "mcmc_checkpoint_size", "mcmc_checkpoint_save",
           "mcmc_checkpoint_load", "mcmc_set_companion", "mcmc_set_twalk", "hmm_posterior",
           "hmm_loglik_grad", "hmm_em_step", "hmm_viterbi", "hmm_simulate", "hmm_validate_params"):
    getattr(_lib, _f).restype = ctypes.c_int


class HMMError(RuntimeError):
    def __init__(self, fn, code):
        super().__init__(f"{fn}: {_lib.hmm_status_string(code).decode()} ({code})")
        self.code = code


def _check(fn, code):
    if code != HMM_OK:
        raise HMMError(fn, code)


def lib():
    return _lib


PARAM_CHECKS = {0: "ok", 1: "delta", 2: "Gamma", 3: "p", 4: "mu", 5: "Sigma"}


def validate_params(delta, Gamma, p, mu, Sigma, tol=0.0):
    """Host check of one parameter set (hmm_validate_params): returns None when
    it is valid, else the name of the first failing block."""
    arrs = [np.ascontiguousarray(np.asarray(a, dtype=np.float64)) for a in (delta, Gamma, p, mu, Sigma)]
    K = arrs[0].size
    sizes = (K, K * K, K, 2 * K, 3 * K)
    if any(a.size != n for a, n in zip(arrs, sizes)):
        raise ValueError("parameter arrays must have K, K*K, K, 2K and 3K entries")
    what = ctypes.c_int32(0)
    rc = _lib.hmm_validate_params(K, *[a.ctypes.data for a in arrs], float(tol), ctypes.byref(what))
    if rc == HMM_OK:
        return None
    if what.value == 0:
        _check("hmm_validate_params", rc)
    return PARAM_CHECKS[what.value]


def _dev(t, dtype, name, numel=None):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be on a GPU")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements, got {t.numel()}")
    return t.data_ptr() if t.numel() else None


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


def loglik_noalloc(delta, Gamma, p, mu, Sigma, flag, xy, algo="blocked_f32", out=None, stream=None):
    """ln L (eq. 2) through hmm_loglik_noalloc (no context, no device allocation
    by the library; the tensors' device must be the current one).  `out` must
    be given where the caller cannot allocate either."""
    K = int(delta.numel())
    T = int(flag.numel())
    if out is None:
        out = torch.empty(1, dtype=torch.float64, device=delta.device)
    a = ALGOS[algo] if isinstance(algo, str) else int(algo)
    rc = _lib.hmm_loglik_noalloc(K, _dev(delta, torch.float64, "delta", K),
                                 _dev(Gamma, torch.float64, "Gamma", K * K),
                                 _dev(p, torch.float64, "p", K), _dev(mu, torch.float64, "mu", 2 * K),
                                 _dev(Sigma, torch.float64, "Sigma", 3 * K), T,
                                 _dev(flag, torch.uint8, "flag", T), _dev(xy, torch.float64, "xy", 2 * T),
                                 a, _stream(stream), _dev(out, torch.float64, "out", 1))
    _check("hmm_loglik_noalloc", rc)
    return out


class Context:
    """One library context (scratch memory, tuning) on one device."""

    def __init__(self, device=0):
        self.device = torch.device("cuda", device) if isinstance(device, int) else torch.device(device)
        h = _vp()
        _check("hmm_ctx_create", _lib.hmm_ctx_create(ctypes.byref(h), self.device.index or 0))
        self._h = h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.hmm_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_blocking(self, block_len=0, fold=0):
        _check("hmm_ctx_set_blocking", _lib.hmm_ctx_set_blocking(self._h, int(block_len), int(fold)))

    def plan(self, K, T):
        L, nb, lv = _i64(), _i64(), _i32()
        _check("hmm_blocked_plan", _lib.hmm_blocked_plan(self._h, int(K), int(T), ctypes.byref(L),
                                                         ctypes.byref(nb), ctypes.byref(lv)))
        return dict(block_len=L.value, n_blocks=nb.value, levels=lv.value)

    def profile(self, on=True):
        """Time the segment-product kernel of blocked calls with HIP events."""
        _check("hmm_ctx_profile", _lib.hmm_ctx_profile(self._h, 1 if on else 0))

    def profile_read(self):
        """(launches, total_ms) of the kernel timed since the last read."""
        n, ms = _i64(), ctypes.c_double()
        _check("hmm_ctx_profile_read", _lib.hmm_ctx_profile_read(self._h, ctypes.byref(n), ctypes.byref(ms)))
        return n.value, ms.value

    def loglik(self, delta, Gamma, p, mu, Sigma, flag, xy, algo="blocked_f32", out=None,
               stream=None):
        """ln L (eq. 2) into a device float64 tensor of one element (returned)."""
        K = int(delta.numel())
        T = int(flag.numel())
        if out is None:
            out = torch.empty(1, dtype=torch.float64, device=delta.device)
        a = ALGOS[algo] if isinstance(algo, str) else int(algo)
        rc = _lib.hmm_loglik(self._h, K, _dev(delta, torch.float64, "delta", K),
                             _dev(Gamma, torch.float64, "Gamma", K * K),
                             _dev(p, torch.float64, "p", K), _dev(mu, torch.float64, "mu", 2 * K),
                             _dev(Sigma, torch.float64, "Sigma", 3 * K), T,
                             _dev(flag, torch.uint8, "flag", T), _dev(xy, torch.float64, "xy", 2 * T),
                             a, _stream(stream), _dev(out, torch.float64, "out", 1))
        _check("hmm_loglik", rc)
        return out

    def loglik_kind(self, kind, delta, Gamma, e0, e1, obs, algo="blocked_f32", out=None, stream=None):
        """ln L (eq. 2) with another emission model: kind 1 Poisson (e0 = lambda, obs int32
        counts), kind 2 1-D Gaussian (e0 = mu, e1 = var, obs float64 values)."""
        K = int(delta.numel())
        T = int(obs.numel())
        if out is None:
            out = torch.empty(1, dtype=torch.float64, device=delta.device)
        a = ALGOS[algo] if isinstance(algo, str) else int(algo)
        obs_t = torch.int32 if int(kind) == EMIS_POISSON else torch.float64
        rc = _lib.hmm_loglik_kind(self._h, int(kind), K, _dev(delta, torch.float64, "delta", K),
                                  _dev(Gamma, torch.float64, "Gamma", K * K), _dev(e0, torch.float64, "e0", K),
                                  _dev(e1, torch.float64, "e1", K) if e1 is not None else None, T,
                                  _dev(obs, obs_t, "obs", T), a, _stream(stream), _dev(out, torch.float64, "out", 1))
        _check("hmm_loglik_kind", rc)
        return out

    def _params(self, delta, Gamma, p, mu, Sigma, flag, xy):
        K = int(delta.numel())
        T = int(flag.numel())
        return K, T, (_dev(delta, torch.float64, "delta", K), _dev(Gamma, torch.float64, "Gamma", K * K),
                      _dev(p, torch.float64, "p", K), _dev(mu, torch.float64, "mu", 2 * K),
                      _dev(Sigma, torch.float64, "Sigma", 3 * K), T,
                      _dev(flag, torch.uint8, "flag", T), _dev(xy, torch.float64, "xy", 2 * T))

    def posterior(self, delta, Gamma, p, mu, Sigma, flag, xy, stats=True, stream=None):
        """State posteriors: dict gamma (T, K) float32, loglik (1,) float64 and, with
        stats, xi (K, K), pre (K,), mom (K, 7) float64 (device tensors)."""
        K, T, args = self._params(delta, Gamma, p, mu, Sigma, flag, xy)
        dev = delta.device
        gamma = torch.empty((T, K), dtype=torch.float32, device=dev)
        st = torch.empty(K * K + 8 * K, dtype=torch.float64, device=dev) if stats else None
        ll = torch.empty(1, dtype=torch.float64, device=dev)
        _check("hmm_posterior", _lib.hmm_posterior(self._h, K, *args, _stream(stream),
                                                   _dev(gamma, torch.float32, "gamma"),
                                                   _dev(st, torch.float64, "stats") if stats else None,
                                                   _dev(ll, torch.float64, "loglik", 1)))
        out = dict(gamma=gamma, loglik=ll)
        if stats:
            out.update(xi=st[:K * K].view(K, K), pre=st[K * K:K * K + K], mom=st[K * K + K:].view(K, 7))
        return out

    def loglik_grad(self, delta, Gamma, p, mu, Sigma, flag, xy, stream=None):
        """(ln L, dict of gradients delta (K,), Gamma (K, K), p (K,), mu (K, 2), Sigma (K, 3))."""
        K, T, args = self._params(delta, Gamma, p, mu, Sigma, flag, xy)
        dev = delta.device
        g = torch.empty(K + K * K + K + 2 * K + 3 * K, dtype=torch.float64, device=dev)
        ll = torch.empty(1, dtype=torch.float64, device=dev)
        _check("hmm_loglik_grad", _lib.hmm_loglik_grad(self._h, K, *args, _stream(stream),
                                                       _dev(ll, torch.float64, "loglik", 1),
                                                       _dev(g, torch.float64, "grad")))
        o = [0, K, K + K * K, 2 * K + K * K, 4 * K + K * K, 7 * K + K * K]
        return ll, dict(delta=g[o[0]:o[1]], Gamma=g[o[1]:o[2]].view(K, K), p=g[o[2]:o[3]],
                        mu=g[o[3]:o[4]].view(K, 2), Sigma=g[o[4]:o[5]].view(K, 3))

    def em_step(self, params, K, flag, xy, out=None, loglik=None, stream=None):
        """One EM iteration from the packed parameters [delta | Gamma | p | mu |
        Sigma] (device float64): returns (new packed parameters, ln L of the
        input).  out=params iterates in place; loglik may be a 1-element view
        (e.g. one entry of a trace) that receives ln L."""
        K = int(K)
        n = K * (K + 7)
        T = int(flag.numel())
        prm = _dev(params, torch.float64, "params", n)
        if out is None:
            out = torch.empty(n, dtype=torch.float64, device=params.device)
        if loglik is None:
            loglik = torch.empty(1, dtype=torch.float64, device=params.device)
        o = [0, K, K + K * K, 2 * K + K * K, 4 * K + K * K]
        _check("hmm_em_step", _lib.hmm_em_step(
            self._h, K, *[prm + 8 * i for i in o], T, _dev(flag, torch.uint8, "flag", T),
            _dev(xy, torch.float64, "xy", 2 * T), _stream(stream), _dev(loglik, torch.float64, "loglik", 1),
            _dev(out, torch.float64, "out", n)))
        return out, loglik

    def viterbi(self, delta, Gamma, p, mu, Sigma, flag, xy, stream=None):
        """Most likely path: (path int32 (T,), first int32 (1,), score float64 (1,)) on the device."""
        K, T, args = self._params(delta, Gamma, p, mu, Sigma, flag, xy)
        dev = delta.device
        path = torch.empty(max(T, 1), dtype=torch.int32, device=dev)
        first = torch.empty(1, dtype=torch.int32, device=dev)
        score = torch.empty(1, dtype=torch.float64, device=dev)
        _check("hmm_viterbi", _lib.hmm_viterbi(self._h, K, *args, _stream(stream),
                                               path.data_ptr() if T else None, first.data_ptr(),
                                               score.data_ptr()))
        return path[:T], first, score

    def simulate(self, K, params, start, H, seed=0, stream=None):
        """Posterior-predictive paths of n draws: dict states (H, n) int32, flags (H, n)
        uint8, xy (H, n, 2) float64, first (n,) int32 (device tensors)."""
        n = int(start.numel()) // int(K)
        dev = start.device
        states = torch.empty((H, n), dtype=torch.int32, device=dev)
        flags = torch.empty((H, n), dtype=torch.uint8, device=dev)
        xy = torch.empty((H, n, 2), dtype=torch.float64, device=dev)
        first = torch.empty(n, dtype=torch.int32, device=dev)
        nh = n * int(H)
        _check("hmm_simulate", _lib.hmm_simulate(
            self._h, n, int(K), _dev(params, torch.float64, "params", n * K * (K + 7)),
            _dev(start, torch.float64, "start", n * K), int(H), int(seed), _stream(stream),
            states.data_ptr() if nh else None, flags.data_ptr() if nh else None, xy.data_ptr() if nh else None,
            first.data_ptr() if n else None))
        return dict(states=states, flags=flags, xy=xy, first=first)

    def batch_graph(self, on=True):
        _check("hmm_ctx_set_batch_graph", _lib.hmm_ctx_set_batch_graph(self._h, 1 if on else 0))

    def set_batch_persistent(self, on=True):
        """Persistent batched segment launches with an atomic job queue (default) or one
        workgroup per job."""
        _check("hmm_ctx_set_batch_persistent", _lib.hmm_ctx_set_batch_persistent(self._h, 1 if on else 0))

    def set_packing(self, mode=1):
        """Segments per wavefront of the FP32 path for 16 < K <= 28: 1 (or True) the
        per-K default, 0 (or False) one segment per wavefront, 2, 4 or 5 column tiles."""
        _check("hmm_ctx_set_packing", _lib.hmm_ctx_set_packing(self._h, int(mode)))

    @staticmethod
    def _desc(K, T, param_off, obs_off):
        import numpy as np
        K = np.ascontiguousarray(K, dtype=np.int32)
        T = np.ascontiguousarray(T, dtype=np.int64)
        param_off = np.ascontiguousarray(param_off, dtype=np.int64)
        obs_off = np.ascontiguousarray(obs_off, dtype=np.int64)
        n = K.shape[0]
        if not (T.shape[0] == param_off.shape[0] == obs_off.shape[0] == n):
            raise ValueError("descriptor arrays must have the same length")
        return n, K, T, param_off, obs_off

    def loglik_batched(self, K, T, param_off, params, obs_off, flag, xy, algo="blocked_f32",
                       out=None, stream=None):
        """ln L of n packed sets (host descriptors K, T, param_off, obs_off; device params,
        flag, xy).  Returns the device float64[n] result."""
        n, K, T, param_off, obs_off = self._desc(K, T, param_off, obs_off)
        if out is None:
            out = torch.empty(n, dtype=torch.float64, device=params.device)
        a = ALGOS[algo] if isinstance(algo, str) else int(algo)
        if xy.numel() != 2 * flag.numel():
            raise ValueError("xy must hold two coordinates per observation")
        rc = _lib.hmm_loglik_batched(self._h, n, K.ctypes.data, T.ctypes.data, param_off.ctypes.data,
                                     _dev(params, torch.float64, "params"), params.numel(),
                                     obs_off.ctypes.data, _dev(flag, torch.uint8, "flag"),
                                     _dev(xy, torch.float64, "xy"), flag.numel(), a, _stream(stream),
                                     _dev(out, torch.float64, "out", n))
        _check("hmm_loglik_batched", rc)
        return out

    def autotune_batched(self, K, T, param_off, params, obs_off, flag, xy, algo="blocked_f32",
                         reps=3):
        """Tune the batched path's segment lengths on these inputs; returns the chosen L per set."""
        import numpy as np
        n, K, T, param_off, obs_off = self._desc(K, T, param_off, obs_off)
        out = torch.empty(n, dtype=torch.float64, device=params.device)
        chosen = np.zeros(n, dtype=np.int64)
        a = ALGOS[algo] if isinstance(algo, str) else int(algo)
        if xy.numel() != 2 * flag.numel():
            raise ValueError("xy must hold two coordinates per observation")
        rc = _lib.hmm_autotune_batched(self._h, n, K.ctypes.data, T.ctypes.data, param_off.ctypes.data,
                                       _dev(params, torch.float64, "params"), params.numel(),
                                       obs_off.ctypes.data, _dev(flag, torch.uint8, "flag"),
                                       _dev(xy, torch.float64, "xy"), flag.numel(), a,
                                       _dev(out, torch.float64, "out", n), int(reps), chosen.ctypes.data)
        _check("hmm_autotune_batched", rc)
        return chosen

    def emission(self, p, mu, Sigma, flag, xy, stream=None):
        """(shift int32[T], e_hat float32[T, K], status int32[1]) of the emission stage."""
        K = int(p.numel())
        T = int(flag.numel())
        shift = torch.empty(T, dtype=torch.int32, device=p.device)
        e_hat = torch.empty((T, K), dtype=torch.float32, device=p.device)
        status = torch.empty(1, dtype=torch.int32, device=p.device)
        rc = _lib.hmm_emission(self._h, K, _dev(p, torch.float64, "p", K),
                               _dev(mu, torch.float64, "mu", 2 * K),
                               _dev(Sigma, torch.float64, "Sigma", 3 * K), T,
                               _dev(flag, torch.uint8, "flag", T), _dev(xy, torch.float64, "xy", 2 * T),
                               _stream(stream), _dev(shift, torch.int32, "shift"),
                               _dev(e_hat, torch.float32, "e_hat"), _dev(status, torch.int32, "status"))
        _check("hmm_emission", rc)
        return shift, e_hat, status


    def theta_to_params(self, K, theta, box, stream=None):
        """(params [n, K(K+7)], logprior [n]) of unconstrained vectors theta [n, K*K+4K]."""
        D = K * K + 4 * K
        n = theta.numel() // D
        if n * D != theta.numel() or n < 1:
            raise ValueError("theta must hold whole vectors of K*K+4K entries")
        params = torch.empty((n, K * (K + 7)), dtype=torch.float64, device=theta.device)
        lp = torch.empty(n, dtype=torch.float64, device=theta.device)
        b = (ctypes.c_double * 4)(*[float(v) for v in box])
        _check("hmm_theta_to_params",
               _lib.hmm_theta_to_params(self._h, int(K), n, _dev(theta, torch.float64, "theta"), b,
                                        _dev(params, torch.float64, "params"), _dev(lp, torch.float64, "lp"),
                                        _stream(stream)))
        return params, lp

    def philox(self, seed, purpose, it, chain, n, normal=False, stream=None):
        """2n draws of Philox counter stream (i, chain, it, purpose), i < n (device float64)."""
        out = torch.empty(2 * max(n, 0), dtype=torch.float64, device=self.device)
        _check("hmm_philox", _lib.hmm_philox(self._h, int(seed), int(purpose), int(it), int(chain), int(n),
                                             1 if normal else 0, _dev(out, torch.float64, "out"),
                                             _stream(stream)))
        return out


MCMC_RANDOM_WALK = 0
MCMC_LEARNED = 1
MCMC_TWALK = 2
# t-walk tuning {p_traverse, p_walk, p_blow, a_t, a_w, n1} (Christen & Fox's defaults)
TWALK_DEFAULT = (0.4918, 0.4918, 0.0082, 6.0, 1.5, 4.0)


class Chains:
    """Parallel Metropolis-Hastings chains over the parameters of a K-state model."""

    def __init__(self, ctx, K, n_chains, flag, xy, box, seed=0, history=1024):
        self.ctx = ctx
        self.K, self.C = int(K), int(n_chains)
        self.D = self.K * self.K + 4 * self.K
        T = int(flag.numel())
        if xy.numel() != 2 * T:
            raise ValueError("xy must hold two coordinates per observation")
        self._obs = (flag, xy)          # keep the observations alive
        b = (ctypes.c_double * 4)(*[float(v) for v in box])
        h = _vp()
        _check("mcmc_create", _lib.mcmc_create(ctx._h, self.K, self.C, T, _dev(flag, torch.uint8, "flag"),
                                               _dev(xy, torch.float64, "xy"), b, int(seed), int(history),
                                               ctypes.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.mcmc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def view(self):
        v = McmcView()
        _check("mcmc_view_get", _lib.mcmc_view_get(self._h, ctypes.byref(v)))
        return v

    def _tensor(self, ptr, shape, dtype):
        """Copy of a library-owned device buffer as a torch tensor (synchronous)."""
        n = 1
        for s in shape:
            n *= s
        out = torch.empty(shape, dtype=dtype, device=self.ctx.device)
        if n:
            torch.cuda.synchronize(self.ctx.device)
            rc = _hip().hipMemcpy(out.data_ptr(), ptr, n * out.element_size(), 3)  # device to device
            if rc != 0:
                raise HMMError("hipMemcpy", HMM_E_DEVICE)
        return out

    def state(self):
        """dict of copies: theta [C, D], loglik [C], logprior [C], accepts [C], iterations."""
        v = self.view()
        return dict(theta=self._tensor(v.theta, (self.C, self.D), torch.float64),
                    loglik=self._tensor(v.loglik, (self.C,), torch.float64),
                    logprior=self._tensor(v.logprior, (self.C,), torch.float64),
                    accepts=self._tensor(v.accepts, (self.C,), torch.int64),
                    iterations=v.iterations)

    def proposal(self):
        """Copies of the last proposals: theta_prop, loglik_prop, logprior_prop, logq_fwd."""
        v = self.view()
        return dict(theta=self._tensor(v.theta_prop, (self.C, self.D), torch.float64),
                    loglik=self._tensor(v.loglik_prop, (self.C,), torch.float64),
                    logprior=self._tensor(v.logprior_prop, (self.C,), torch.float64),
                    logq_fwd=self._tensor(v.logq_fwd, (self.C,), torch.float64))

    def history(self):
        """(states [H, C, D] float32, logpost [H, C] float64, iterations); slot t % H holds iteration t."""
        v = self.view()
        return (self._tensor(v.history, (v.history_len, self.C, self.D), torch.float32),
                self._tensor(v.history_logpost, (v.history_len, self.C), torch.float64), v.iterations)

    def network(self):
        """dict of copies: weights (flat float32), center, in_scale, out_scale, lag, hidden, trained."""
        v = self.view()
        return dict(weights=self._tensor(v.net_weights, (v.net_count,), torch.float32),
                    center=self._tensor(v.center, (self.D,), torch.float64),
                    in_scale=self._tensor(v.in_scale, (self.D,), torch.float64),
                    out_scale=self._tensor(v.out_scale, (self.D,), torch.float64),
                    lag=v.lag, hidden=v.net_hidden, trained=bool(v.trained))

    def set_state(self, theta, rw_scale, stream=None):
        theta = theta.reshape(-1)
        _check("mcmc_set_state", _lib.mcmc_set_state(self._h, _dev(theta, torch.float64, "theta", self.C * self.D),
                                                     _dev(rw_scale, torch.float64, "rw_scale", self.D),
                                                     _stream(stream)))

    def set_companion(self, theta2, stream=None):
        """Second t-walk point of every chain (device [C, D] float64)."""
        theta2 = theta2.reshape(-1)
        _check("mcmc_set_companion", _lib.mcmc_set_companion(
            self._h, _dev(theta2, torch.float64, "theta2", self.C * self.D), _stream(stream)))

    def set_twalk(self, tuning=TWALK_DEFAULT):
        t = (ctypes.c_double * 6)(*[float(v) for v in tuning])
        _check("mcmc_set_twalk", _lib.mcmc_set_twalk(self._h, t))

    def twalk_state(self):
        """dict of copies: theta2 [C, D], loglik2 [C], logprior2 [C], counts [C, 4, 2]
        (proposed, accepted per kernel), code [C] of the last proposal."""
        v = self.view()
        return dict(theta2=self._tensor(v.theta2, (self.C, self.D), torch.float64),
                    loglik2=self._tensor(v.loglik2, (self.C,), torch.float64),
                    logprior2=self._tensor(v.logprior2, (self.C,), torch.float64),
                    counts=self._tensor(v.twalk_counts, (self.C, 4, 2), torch.int64),
                    code=self._tensor(v.twalk_code, (self.C,), torch.int32),
                    companion=bool(v.companion))

    def set_rw_scale(self, rw_scale, stream=None):
        _check("mcmc_set_rw_scale", _lib.mcmc_set_rw_scale(
            self._h, _dev(rw_scale, torch.float64, "rw_scale", self.D), _stream(stream)))

    def step(self, n_iter=1, proposal=MCMC_RANDOM_WALK, eps=0.1, stream=None):
        _check("mcmc_step", _lib.mcmc_step(self._h, int(n_iter), int(proposal), float(eps), _stream(stream)))

    def train(self, steps, batch=256, lag=1, lr=1e-3, window=0, weight_decay=0.0, window_end=0, holdout=0.0,
              val_every=25, val_batch=512, stream=None, losses=True):
        """Train the proposal network on lagged pairs of the history.

        Returns a dict: ``loss`` (device float32[steps], minibatch losses) and, with
        holdout > 0, ``val`` (device held-out losses, the first before any step) and
        ``best_step`` (Adam step whose weights were kept, -1 = the starting weights)."""
        o = TrainOpts(int(steps), int(batch), int(lag), float(lr), float(weight_decay), int(window),
                      int(window_end), float(holdout), int(val_every), int(val_batch))
        out = torch.empty(max(steps, 1), dtype=torch.float32, device=self.ctx.device) if losses else None
        n_val = 1 + (-(-steps // max(int(val_every), 1))) if holdout > 0 else 0
        val = torch.empty(max(n_val, 1), dtype=torch.float32, device=self.ctx.device) if n_val else None
        best = _i32(-2)
        _check("mcmc_train_proposal", _lib.mcmc_train_proposal(
            self._h, ctypes.byref(o), _stream(stream), _dev(out, torch.float32, "loss") if losses else None,
            _dev(val, torch.float32, "val") if n_val else None, ctypes.byref(best) if n_val else None))
        return dict(loss=out[:steps] if losses else None, val=val[:n_val] if n_val else None,
                    best_step=best.value if n_val else None)

    def reset_proposal(self, seed=0, stream=None):
        _check("mcmc_reset_proposal", _lib.mcmc_reset_proposal(self._h, int(seed), _stream(stream)))

    def mlp_forward(self, X, stream=None):
        n = X.numel() // self.D
        out = torch.empty((n, 2 * self.D), dtype=torch.float32, device=X.device)
        _check("mlp_forward", _lib.mlp_forward(self._h, n, _dev(X, torch.float32, "X", n * self.D),
                                               _dev(out, torch.float32, "out"), _stream(stream)))
        return out

    def mlp_loss_grad(self, X, R, stream=None):
        n = X.numel() // self.D
        v = self.view()
        rows = torch.empty(n, dtype=torch.float32, device=X.device)
        grad = torch.empty(v.net_count, dtype=torch.float32, device=X.device)
        _check("mlp_loss_grad", _lib.mlp_loss_grad(self._h, n, _dev(X, torch.float32, "X", n * self.D),
                                                   _dev(R, torch.float32, "R", n * self.D),
                                                   _dev(rows, torch.float32, "row_loss"),
                                                   _dev(grad, torch.float32, "grad"), _stream(stream)))
        return rows, grad

    def checkpoint(self, stream=None):
        """The sampler's checkpoint image (bytes)."""
        n = _i64()
        _check("mcmc_checkpoint_size", _lib.mcmc_checkpoint_size(self._h, ctypes.byref(n)))
        buf = ctypes.create_string_buffer(n.value)
        _check("mcmc_checkpoint_save", _lib.mcmc_checkpoint_save(self._h, buf, n.value, _stream(stream)))
        return buf.raw

    def restore(self, image, stream=None):
        """Continue from a checkpoint image made by `checkpoint`."""
        buf = ctypes.create_string_buffer(bytes(image), len(image))
        _check("mcmc_checkpoint_load", _lib.mcmc_checkpoint_load(self._h, buf, len(image), _stream(stream)))

    def set_network(self, weights, center, in_scale, out_scale, lag, stream=None):
        v = self.view()
        _check("mlp_set_weights", _lib.mlp_set_weights(
            self._h, _dev(weights, torch.float32, "weights", v.net_count),
            _dev(center, torch.float64, "center", self.D), _dev(in_scale, torch.float64, "in_scale", self.D),
            _dev(out_scale, torch.float64, "out_scale", self.D), int(lag), _stream(stream)))


_hip_lib = None


def _hip():
    """The HIP runtime, for copies out of library-owned buffers."""
    global _hip_lib
    if _hip_lib is None:
        _hip_lib = ctypes.CDLL("libamdhip64.so")
        _hip_lib.hipMemcpy.argtypes = [_vp, _vp, ctypes.c_size_t, ctypes.c_int]
        _hip_lib.hipMemcpy.restype = ctypes.c_int
    return _hip_lib


def batch_to_device(packed, device="cuda"):
    """Device tensors for a packed batch (synth.pack / synth.batch)."""
    return dict(K=packed["K"], T=packed["T"], param_off=packed["param_off"], obs_off=packed["obs_off"],
                params=torch.as_tensor(packed["params"], dtype=torch.float64, device=device).contiguous(),
                flag=torch.as_tensor(packed["flag"], dtype=torch.uint8, device=device).contiguous(),
                xy=torch.as_tensor(packed["xy"], dtype=torch.float64, device=device).contiguous())


def to_device(prm, obs, device="cuda"):
    """Move a synth (HMMParams, Observations) pair to device tensors."""
    f64 = dict(dtype=torch.float64, device=device)
    return dict(delta=torch.as_tensor(prm.delta, **f64).contiguous(),
                Gamma=torch.as_tensor(prm.Gamma, **f64).contiguous(),
                p=torch.as_tensor(prm.p, **f64).contiguous(),
                mu=torch.as_tensor(prm.mu, **f64).contiguous(),
                Sigma=torch.as_tensor(prm.Sigma, **f64).contiguous(),
                flag=torch.as_tensor(obs.flag, dtype=torch.uint8, device=device).contiguous(),
                xy=torch.as_tensor(obs.xy, **f64).contiguous())


def kind_to_device(ks, device="cuda"):
    """Device tensors for a synth.KindSet (delta, Gamma, e0, e1, obs)."""
    f64 = dict(dtype=torch.float64, device=device)
    obs_t = torch.int32 if ks.kind == EMIS_POISSON else torch.float64
    return dict(delta=torch.as_tensor(ks.delta, **f64).contiguous(),
                Gamma=torch.as_tensor(ks.Gamma, **f64).contiguous(),
                e0=torch.as_tensor(ks.e0, **f64).contiguous(),
                e1=torch.as_tensor(ks.e1, **f64).contiguous(),
                obs=torch.as_tensor(ks.obs, dtype=obs_t, device=device).contiguous())
