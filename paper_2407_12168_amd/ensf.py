"""Python binding of libensf (the C ABI in include/ensf.h), argument marshalling only.

Every function has the name of the C entry point it calls.  Arrays are torch tensors on
the context's GPU (float32 / int32, contiguous); torch provides device memory and the
stream, every step of the analysis runs in the library's HIP kernels.  If the shared
library has not been built, every call raises EnsfError.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libensf.so")
# tile shapes measured by ensf_autotune on MI355X for the benchmark shapes
DEFAULT_TUNE_CACHE = os.path.join(HERE, "tune_gfx950.json")

(ENSF_OK, ENSF_EINVAL, ENSF_ENOMEM, ENSF_EHIP, ENSF_ENONFINITE, ENSF_EUNSUPPORTED,
 ENSF_ESCRATCH) = range(7)
NOALLOC_SCRATCH_BYTES = 64 << 20   # ENSF_NOALLOC_SCRATCH_BYTES
PRECISIONS = {"fp32": 0, "bf16x3": 1, "bf16": 2}
OBS_OPS = {"arctan": 0, "linear": 1}
LIK_STEPS = {"explicit": 0, "implicit": 1}
INIT_STEP = 0xFFFFFFFF


class EnsfError(RuntimeError):
    def __init__(self, status, what=""):
        self.status = status
        msg = _lib().ensf_status_string(status).decode() if _LIB is not None else str(status)
        if _LIB is not None and status in (ENSF_EHIP, ENSF_ENOMEM):
            msg += f" [{_LIB.ensf_last_error_string().decode()}]"
        super().__init__(f"{what}: {msg} (status {status})" if what else msg)


class ensf_options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("obs_op", ctypes.c_int32),
                ("eps_alpha", ctypes.c_double), ("spread_relax", ctypes.c_double),
                ("use_graph", ctypes.c_int32), ("device", ctypes.c_int32),
                ("tune_cache", ctypes.c_char_p), ("lik_step", ctypes.c_int32),
                ("wx_sparse", ctypes.c_int32)]


class ensf_problem(ctypes.Structure):
    _fields_ = [("d_prior", ctypes.c_void_p), ("n_members", ctypes.c_int32),
                ("dim", ctypes.c_int64), ("d_post", ctypes.c_void_p),
                ("n_particles", ctypes.c_int32), ("d_obs_idx", ctypes.c_void_p),
                ("d_obs_val", ctypes.c_void_p), ("n_obs", ctypes.c_int64),
                ("obs_sigma", ctypes.c_float), ("n_steps", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("filter_id", ctypes.c_uint32)]


_LIB = None
EXPORTS = ("ensf_default_options", "ensf_create", "ensf_analysis", "ensf_analysis_batched",
           "ensf_score", "ensf_rng_normal", "ensf_ensemble_stats", "ensf_sync_status",
           "ensf_autotune", "ensf_autotune_batched", "ensf_profile_phases", "ensf_phase_times",
           "ensf_destroy", "ensf_status_string", "ensf_last_error_string",
           "ensf_analysis_noalloc", "ensf_measure_mfma_rate")


def _lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise EnsfError(ENSF_EUNSUPPORTED, f"{LIB_PATH} is not built "
                            "(run python -m paper_2407_12168_amd.build)")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, u32, u64 = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                                  ctypes.c_uint32, ctypes.c_uint64)
        L.ensf_default_options.argtypes = [ctypes.POINTER(ensf_options)]
        L.ensf_default_options.restype = None
        L.ensf_create.argtypes = [ctypes.POINTER(ensf_options), ctypes.POINTER(vp)]
        L.ensf_analysis.argtypes = [vp, vp, i32, i64, vp, i32, vp, vp, i64, ctypes.c_float, i32,
                                    u64, u32, vp]
        L.ensf_analysis_batched.argtypes = [vp, ctypes.POINTER(ensf_problem), i32, vp]
        L.ensf_score.argtypes = [vp, vp, i32, i64, vp, i32, vp, vp, i64, ctypes.c_float,
                                 ctypes.c_double, vp, vp, vp]
        L.ensf_rng_normal.argtypes = [u64, u32, u32, u32, i64, vp, vp, vp]
        L.ensf_ensemble_stats.argtypes = [vp, i32, i64, vp, vp, vp]
        L.ensf_sync_status.argtypes = [vp, ctypes.POINTER(i64)]
        L.ensf_autotune.argtypes = [vp, ctypes.POINTER(ensf_problem), vp]
        L.ensf_autotune_batched.argtypes = [vp, ctypes.POINTER(ensf_problem), i32, vp]
        L.ensf_profile_phases.argtypes = [vp, i32]
        L.ensf_phase_times.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64)]
        L.ensf_destroy.argtypes = [vp]
        L.ensf_analysis_noalloc.argtypes = [ctypes.POINTER(ensf_options), vp, i32, i64, vp, i32,
                                            vp, vp, i64, ctypes.c_float, i32, u64, u32, vp, vp]
        L.ensf_measure_mfma_rate.argtypes = [i32, ctypes.POINTER(ctypes.c_double), vp]
        L.ensf_status_string.argtypes = [ctypes.c_int]
        L.ensf_status_string.restype = ctypes.c_char_p
        L.ensf_last_error_string.argtypes = []
        L.ensf_last_error_string.restype = ctypes.c_char_p
        for name in EXPORTS:
            if name not in ("ensf_default_options", "ensf_status_string",
                            "ensf_last_error_string"):
                getattr(L, name).restype = ctypes.c_int
        _LIB = L
    return _LIB


def _check(status, what):
    if status != ENSF_OK:
        raise EnsfError(status, what)


def _ptr(t, dtype=None, name="tensor"):
    if t is None:
        return None
    if not t.is_cuda:
        raise EnsfError(ENSF_EINVAL, f"{name} must be a GPU tensor")
    if not t.is_contiguous():
        raise EnsfError(ENSF_EINVAL, f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise EnsfError(ENSF_EINVAL, f"{name} must be {dtype}")
    return t.data_ptr()


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def _obs(obs_idx, obs_val):
    import torch
    if obs_idx is None or obs_idx.numel() == 0:
        return None, None, 0
    if obs_val is None or obs_val.numel() != obs_idx.numel():
        raise EnsfError(ENSF_EINVAL, "obs_idx and obs_val differ in length")
    return (_ptr(obs_idx, torch.int32, "obs_idx"), _ptr(obs_val, torch.float32, "obs_val"),
            obs_idx.numel())


def ensf_default_options():
    o = ensf_options()
    _lib().ensf_default_options(ctypes.byref(o))
    return o


def ensf_create(precision="fp32", obs_op="arctan", eps_alpha=0.05, spread_relax=0.0,
                use_graph=True, device=0, tune_cache=DEFAULT_TUNE_CACHE, lik_step="explicit",
                wx_sparse=False):
    o = make_options(precision, obs_op, eps_alpha, spread_relax, use_graph, device, tune_cache,
                     lik_step, wx_sparse)
    h = ctypes.c_void_p()
    _check(_lib().ensf_create(ctypes.byref(o), ctypes.byref(h)), "ensf_create")
    return h


def ensf_analysis(ctx, prior, post, obs_idx, obs_val, obs_sigma, n_steps, seed, filter_id=0,
                  stream=None):
    import torch
    N, d = prior.shape
    idx, val, m = _obs(obs_idx, obs_val)
    _check(_lib().ensf_analysis(ctx, _ptr(prior, torch.float32, "prior"), N, d,
                                _ptr(post, torch.float32, "post"), post.shape[0], idx, val, m,
                                float(obs_sigma), int(n_steps), int(seed), int(filter_id),
                                _stream(stream)), "ensf_analysis")


def make_options(precision="fp32", obs_op="arctan", eps_alpha=0.05, spread_relax=0.0,
                 use_graph=True, device=0, tune_cache=None, lik_step="explicit",
                 wx_sparse=False):
    o = ensf_default_options()
    o.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    o.obs_op = OBS_OPS[obs_op] if isinstance(obs_op, str) else int(obs_op)
    o.eps_alpha = eps_alpha
    o.spread_relax = spread_relax
    # True/False, or the ensf_options value: 0 eager, 1 or 3 graph, 2 one cooperative launch
    # (persistent pseudo-time loop) when the tiles allow it
    o.use_graph = int(use_graph) if not isinstance(use_graph, bool) else (1 if use_graph else 0)
    o.device = device
    o.tune_cache = tune_cache.encode() if tune_cache else None
    o.lik_step = LIK_STEPS[lik_step] if isinstance(lik_step, str) else int(lik_step)
    o.wx_sparse = 1 if wx_sparse else 0
    return o


def ensf_analysis_noalloc(prior, post, obs_idx, obs_val, obs_sigma, n_steps, seed, filter_id=0,
                          counters=None, stream=None, **options):
    """Context-free analysis in the library's static scratch buffer (no allocation).
    counters: None or an int64 GPU tensor of 2 elements that the call adds to (non-finite
    particle values, invalid observations).  options: as ensf_create."""
    import torch
    N, d = prior.shape
    idx, val, m = _obs(obs_idx, obs_val)
    o = make_options(**options)
    _check(_lib().ensf_analysis_noalloc(ctypes.byref(o), _ptr(prior, torch.float32, "prior"), N,
                                        d, _ptr(post, torch.float32, "post"), post.shape[0], idx,
                                        val, m, float(obs_sigma), int(n_steps), int(seed),
                                        int(filter_id),
                                        _ptr(counters, torch.int64, "counters"),
                                        _stream(stream)), "ensf_analysis_noalloc")


def make_problem(prior, post, obs_idx, obs_val, obs_sigma, n_steps, seed, filter_id=0):
    import torch
    idx, val, m = _obs(obs_idx, obs_val)
    p = ensf_problem()
    p.d_prior = _ptr(prior, torch.float32, "prior")
    p.n_members, p.dim = prior.shape
    p.d_post = _ptr(post, torch.float32, "post")
    p.n_particles = post.shape[0]
    p.d_obs_idx, p.d_obs_val, p.n_obs = idx, val, m
    p.obs_sigma = float(obs_sigma)
    p.n_steps = int(n_steps)
    p.seed = int(seed)
    p.filter_id = int(filter_id)
    return p


def ensf_analysis_batched(ctx, problems, stream=None):
    arr = (ensf_problem * len(problems))(*problems)
    _check(_lib().ensf_analysis_batched(ctx, arr, len(problems), _stream(stream)),
           "ensf_analysis_batched")


def ensf_score(ctx, prior, z, obs_idx, obs_val, obs_sigma, t, score, weights=None, stream=None):
    import torch
    N, d = prior.shape
    idx, val, m = _obs(obs_idx, obs_val)
    _check(_lib().ensf_score(ctx, _ptr(prior, torch.float32, "prior"), N, d,
                             _ptr(z, torch.float32, "z"), z.shape[0], idx, val, m,
                             float(obs_sigma), float(t), _ptr(score, torch.float32, "score"),
                             _ptr(weights, torch.float32, "weights"), _stream(stream)),
           "ensf_score")


def ensf_rng_normal(seed, filter_id, step, particle, out, raw=None, stream=None):
    import torch
    _check(_lib().ensf_rng_normal(int(seed), int(filter_id), int(step), int(particle),
                                  out.numel(), _ptr(out, torch.float32, "out"),
                                  _ptr(raw, torch.int32, "raw") if raw is not None else None,
                                  _stream(stream)), "ensf_rng_normal")


def ensf_ensemble_stats(ens, mean, spread, stream=None):
    import torch
    n, d = ens.shape
    _check(_lib().ensf_ensemble_stats(_ptr(ens, torch.float32, "ens"), n, d,
                                      _ptr(mean, torch.float32, "mean"),
                                      _ptr(spread, torch.float32, "spread"), _stream(stream)),
           "ensf_ensemble_stats")


def ensf_sync_status(ctx):
    """Returns (status, nonfinite_count) without raising."""
    n = ctypes.c_int64(0)
    st = _lib().ensf_sync_status(ctx, ctypes.byref(n))
    return st, n.value


def ensf_autotune(ctx, problem, stream=None):
    _check(_lib().ensf_autotune(ctx, ctypes.byref(problem), _stream(stream)), "ensf_autotune")


def ensf_autotune_batched(ctx, problems, stream=None):
    arr = (ensf_problem * len(problems))(*problems)
    _check(_lib().ensf_autotune_batched(ctx, arr, len(problems), _stream(stream)),
           "ensf_autotune_batched")


def ensf_profile_phases(ctx, enable):
    _check(_lib().ensf_profile_phases(ctx, 1 if enable else 0), "ensf_profile_phases")


def ensf_phase_times(ctx):
    """(gram_ms, softmax_ms, wx_ms) summed over profiled pseudo-steps, and that step count."""
    ms = (ctypes.c_double * 3)()
    n = ctypes.c_int64(0)
    _check(_lib().ensf_phase_times(ctx, ms, ctypes.byref(n)), "ensf_phase_times")
    return tuple(ms), n.value


def ensf_measure_mfma_rate(precision="bf16x3", stream=None):
    """Attainable dense MFMA TFLOP/s of the current device for a form's matrix instruction."""
    out = ctypes.c_double(0.0)
    _check(_lib().ensf_measure_mfma_rate(PRECISIONS[precision], ctypes.byref(out),
                                         _stream(stream)), "ensf_measure_mfma_rate")
    return out.value


def ensf_destroy(ctx):
    if ctx is not None and ctx.value:
        _check(_lib().ensf_destroy(ctx), "ensf_destroy")


class Context:
    """Owns one ensf_ctx; destroy() is idempotent."""

    def __init__(self, **opts):
        self.handle = ensf_create(**opts)

    def destroy(self):
        h, self.handle = self.handle, None
        if h is not None:
            ensf_destroy(h)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.destroy()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass
