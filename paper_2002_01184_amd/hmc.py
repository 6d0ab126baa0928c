"""ctypes binding of libhmc.so (include/hmc.h).

Argument marshalling only: every step of the sampler runs in the HIP kernels
of libhmc.so.  The functions keep the C names (hmc_init, hmc_step,
hmc_sample_chain, ...); `Sampler` is a small convenience wrapper that owns a
PyTorch workspace tensor and passes torch's current HIP stream.

Loading fails loudly (RuntimeError) when libhmc.so has not been built: there
is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
# HMC_LIB_PATH selects another build of the same library (the sanitizer build of
# the host runtime); there is no fallback when the file is missing.
LIB_PATH = os.environ.get("HMC_LIB_PATH") or os.path.join(_HERE, "libhmc.so")

# hmc_status
HMC_OK, HMC_E_INVALID, HMC_E_UNSUPPORTED, HMC_E_NOMEM, HMC_E_DEVICE, HMC_E_BUSY = range(6)
# hmc_dtype
HMC_F64, HMC_F32, HMC_BF16 = 0, 1, 2
# hmc_target_kind
HMC_TGT_STD_NORMAL, HMC_TGT_GAUSS_DIAG, HMC_TGT_GAUSS_DENSE, HMC_TGT_LOGREG = 0, 1, 2, 3
# forms
HMC_FORM_AUTO, HMC_FORM_PLAIN, HMC_FORM_FUSED, HMC_FORM_GRAPH = 0, 1, 2, 3
FORM_NAMES = {HMC_FORM_PLAIN: "plain", HMC_FORM_FUSED: "fused", HMC_FORM_GRAPH: "graph"}


class hmc_target(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("reserved0", ctypes.c_int32), ("dim", ctypes.c_int64),
                ("prec", ctypes.c_void_p), ("X", ctypes.c_void_p), ("x_dtype", ctypes.c_int32),
                ("reserved1", ctypes.c_int32), ("n_rows", ctypes.c_int64), ("y", ctypes.c_void_p),
                ("prior_scale", ctypes.c_double)]


class hmc_config(ctypes.Structure):
    _fields_ = [("num_chains", ctypes.c_int64), ("num_leapfrog_steps", ctypes.c_int32),
                ("state_dtype", ctypes.c_int32), ("grad_dtype", ctypes.c_int32), ("form", ctypes.c_int32),
                ("seed", ctypes.c_uint64)]


HMC_ADAPT_DUAL_AVERAGING, HMC_ADAPT_SIMPLE = 0, 1


class hmc_adapt(ctypes.Structure):
    _fields_ = [("enabled", ctypes.c_int32), ("kind", ctypes.c_int32), ("target_accept", ctypes.c_double),
                ("gamma", ctypes.c_double), ("t0", ctypes.c_double), ("kappa", ctypes.c_double),
                ("rate", ctypes.c_double)]


def make_adapt(adapt, target_accept=0.8, gamma=0.05, t0=10.0, kappa=0.75, rate=0.01):
    """adapt: False / None (fixed step), True or "dual_averaging", "simple"."""
    if adapt is False or adapt is None:
        return None
    if adapt is True or adapt == "dual_averaging":
        kind = HMC_ADAPT_DUAL_AVERAGING
    elif adapt == "simple":
        kind = HMC_ADAPT_SIMPLE
    else:
        raise ValueError(f"unknown adaptation {adapt!r}")
    return hmc_adapt(1, kind, target_accept, gamma, t0, kappa, rate)


class hmc_moments(ctypes.Structure):
    _fields_ = [("mean", ctypes.c_void_p), ("m2", ctypes.c_void_p), ("batch_sum", ctypes.c_void_p),
                ("batch_len", ctypes.c_int64), ("ring", ctypes.c_void_p), ("ring_rows", ctypes.c_int64)]


class hmc_trace(ctypes.Structure):
    _fields_ = [("step_size", ctypes.c_void_p), ("is_accepted", ctypes.c_void_p),
                ("log_accept_ratio", ctypes.c_void_p), ("target_log_prob", ctypes.c_void_p)]


class hmc_step_out(ctypes.Structure):
    _fields_ = [("is_accepted", ctypes.c_void_p), ("log_accept_ratio", ctypes.c_void_p),
                ("target_log_prob", ctypes.c_void_p), ("proposed_state", ctypes.c_void_p),
                ("proposed_momentum", ctypes.c_void_p), ("delta_h", ctypes.c_void_p)]


class hmc_request(ctypes.Structure):
    _fields_ = [("target", hmc_target), ("config", hmc_config), ("init_state", ctypes.c_void_p),
                ("step_size", ctypes.c_double), ("num_results", ctypes.c_int64), ("num_burnin", ctypes.c_int64),
                ("adapt", hmc_adapt), ("samples", ctypes.c_void_p), ("trace", hmc_trace)]


class hmc_server_stats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in ("submitted", "admitted", "completed", "failed", "active", "pending",
                                              "ticks", "batched_launches", "max_active")] + \
               [(n, ctypes.c_size_t) for n in ("pool_bytes", "bytes_in_use", "peak_bytes_in_use")] + \
               [("batched_plain_transitions", ctypes.c_int64)]


HMC_REQ_QUEUED, HMC_REQ_RUNNING, HMC_REQ_DONE, HMC_REQ_FAILED = range(4)

EXPORTED = ["hmc_workspace_size", "hmc_init", "hmc_step", "hmc_sample_chain", "hmc_get_state", "hmc_set_state",
            "hmc_destroy", "hmc_last_error", "hmc_effective_form", "hmc_autotune", "hmc_set_inverse_temperature",
            "hmc_remc_swap", "hmc_remc_sample_chain", "hmc_sample_chain_moments", "hmc_set_transform_scale",
            "hmc_nuts_workspace_size", "hmc_nuts_sample_chain", "hmc_server_create", "hmc_server_submit",
            "hmc_server_poll", "hmc_server_wait", "hmc_server_take", "hmc_server_get_stats",
            "hmc_server_destroy", "hmc_sample_chain_noalloc", "hmc_kernel_timer_start", "hmc_kernel_timer_read",
            "hmc_peak_memory", "hmc_peak_compute"]

HMC_NOALLOC_WORKSPACE_BYTES = 64 << 20

_lib = None


def lib():
    """Load libhmc.so (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libhmc.so not built ({LIB_PATH}); run `python -m paper_2002_01184_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp, st = ctypes.c_void_p, ctypes.c_int
    L.hmc_workspace_size.argtypes = [ctypes.POINTER(hmc_target), ctypes.POINTER(hmc_config),
                                     ctypes.POINTER(ctypes.c_size_t)]
    L.hmc_workspace_size.restype = st
    L.hmc_init.argtypes = [ctypes.POINTER(hmc_target), ctypes.POINTER(hmc_config), vp,
                           ctypes.POINTER(ctypes.c_double), ctypes.c_int64, vp, ctypes.c_size_t, vp,
                           ctypes.POINTER(vp)]
    L.hmc_init.restype = st
    L.hmc_step.argtypes = [vp, ctypes.POINTER(hmc_step_out)]
    L.hmc_step.restype = st
    L.hmc_sample_chain.argtypes = [vp, ctypes.c_int64, ctypes.c_int64, ctypes.POINTER(hmc_adapt), vp,
                                   ctypes.POINTER(hmc_trace)]
    L.hmc_sample_chain.restype = st
    L.hmc_get_state.argtypes = [vp, vp, vp, ctypes.POINTER(ctypes.c_uint64)]
    L.hmc_get_state.restype = st
    L.hmc_set_state.argtypes = [vp, vp, vp, ctypes.c_uint64]
    L.hmc_set_state.restype = st
    L.hmc_destroy.argtypes = [vp]
    L.hmc_destroy.restype = st
    L.hmc_sample_chain_noalloc.argtypes = [ctypes.POINTER(hmc_target), ctypes.POINTER(hmc_config), vp,
                                           ctypes.POINTER(ctypes.c_double), ctypes.c_int64, ctypes.c_int64,
                                           ctypes.c_int64, ctypes.POINTER(hmc_adapt), vp, ctypes.POINTER(hmc_trace),
                                           vp, vp, vp]
    L.hmc_sample_chain_noalloc.restype = st
    L.hmc_kernel_timer_start.argtypes = [vp, ctypes.c_int64]
    L.hmc_kernel_timer_start.restype = st
    L.hmc_kernel_timer_read.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64),
                                        ctypes.c_char_p, ctypes.c_size_t]
    L.hmc_kernel_timer_read.restype = st
    L.hmc_last_error.argtypes = []
    L.hmc_last_error.restype = ctypes.c_char_p
    L.hmc_effective_form.argtypes = [vp]
    L.hmc_effective_form.restype = ctypes.c_int32
    L.hmc_autotune.argtypes = [vp, ctypes.c_int32, ctypes.c_char_p, ctypes.c_size_t]
    L.hmc_autotune.restype = st
    L.hmc_sample_chain_moments.argtypes = [vp, ctypes.c_int64, ctypes.c_int64, ctypes.POINTER(hmc_adapt),
                                           ctypes.POINTER(hmc_moments), ctypes.POINTER(hmc_trace)]
    L.hmc_sample_chain_moments.restype = st
    L.hmc_nuts_workspace_size.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)]
    L.hmc_nuts_workspace_size.restype = st
    L.hmc_nuts_sample_chain.argtypes = [vp, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64,
                                        ctypes.POINTER(hmc_adapt), vp, ctypes.c_size_t, vp, vp, vp, vp]
    L.hmc_nuts_sample_chain.restype = st
    L.hmc_set_transform_scale.argtypes = [vp, vp]
    L.hmc_set_transform_scale.restype = st
    L.hmc_set_inverse_temperature.argtypes = [vp, vp]
    L.hmc_set_inverse_temperature.restype = st
    L.hmc_remc_swap.argtypes = [vp, ctypes.c_int64, ctypes.c_uint64, vp]
    L.hmc_remc_swap.restype = st
    L.hmc_remc_sample_chain.argtypes = [vp, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                                        ctypes.POINTER(hmc_adapt), vp, ctypes.POINTER(hmc_trace), vp]
    L.hmc_remc_sample_chain.restype = st
    L.hmc_server_create.argtypes = [ctypes.c_size_t, ctypes.c_int32, ctypes.POINTER(vp)]
    L.hmc_server_create.restype = st
    L.hmc_server_submit.argtypes = [vp, ctypes.POINTER(hmc_request), ctypes.POINTER(ctypes.c_uint64)]
    L.hmc_server_submit.restype = st
    for n in ("hmc_server_poll", "hmc_server_wait"):
        getattr(L, n).argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double)]
        getattr(L, n).restype = st
    L.hmc_server_take.argtypes = [vp, ctypes.c_uint64, vp]
    L.hmc_server_take.restype = st
    L.hmc_server_get_stats.argtypes = [vp, ctypes.POINTER(hmc_server_stats)]
    L.hmc_server_get_stats.restype = st
    L.hmc_server_destroy.argtypes = [vp]
    L.hmc_server_destroy.restype = st
    L.hmc_peak_memory.argtypes = [vp, ctypes.c_size_t, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, vp,
                                  ctypes.POINTER(ctypes.c_double)]
    L.hmc_peak_memory.restype = st
    L.hmc_peak_compute.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, vp,
                                   ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
    L.hmc_peak_compute.restype = st
    _lib = L
    return L


class HMCError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"hmc status {status}: {msg}")
        self.status = status


def _check(status: int):
    if status != HMC_OK:
        raise HMCError(status, lib().hmc_last_error().decode())


# ---- C entry points under their own names --------------------------------
def hmc_workspace_size(target: hmc_target, config: hmc_config) -> int:
    n = ctypes.c_size_t(0)
    _check(lib().hmc_workspace_size(ctypes.byref(target), ctypes.byref(config), ctypes.byref(n)))
    return n.value


def hmc_init(target, config, init_state_ptr, step_sizes, workspace_ptr, workspace_bytes, stream_ptr):
    arr = (ctypes.c_double * len(step_sizes))(*[float(v) for v in step_sizes])
    ctx = ctypes.c_void_p()
    _check(lib().hmc_init(ctypes.byref(target), ctypes.byref(config), init_state_ptr, arr, len(step_sizes),
                          workspace_ptr, workspace_bytes, stream_ptr, ctypes.byref(ctx)))
    return ctx


def hmc_step(ctx, out: hmc_step_out | None = None):
    _check(lib().hmc_step(ctx, ctypes.byref(out) if out is not None else None))


def hmc_sample_chain(ctx, num_results, num_burnin_steps, adapt: hmc_adapt | None, samples_ptr,
                     trace: hmc_trace | None):
    _check(lib().hmc_sample_chain(ctx, num_results, num_burnin_steps,
                                  ctypes.byref(adapt) if adapt is not None else None, samples_ptr,
                                  ctypes.byref(trace) if trace is not None else None))


def hmc_sample_chain_noalloc(target, config, init_state_ptr, step_sizes, num_results, num_burnin_steps,
                             adapt: hmc_adapt | None, samples_ptr, trace: hmc_trace | None, final_state_ptr,
                             final_step_size_ptr, stream_ptr):
    arr = (ctypes.c_double * len(step_sizes))(*[float(v) for v in step_sizes])
    _check(lib().hmc_sample_chain_noalloc(ctypes.byref(target), ctypes.byref(config), init_state_ptr, arr,
                                          len(step_sizes), num_results, num_burnin_steps,
                                          ctypes.byref(adapt) if adapt is not None else None, samples_ptr,
                                          ctypes.byref(trace) if trace is not None else None, final_state_ptr,
                                          final_step_size_ptr, stream_ptr))


def hmc_kernel_timer_start(ctx, max_launches: int):
    _check(lib().hmc_kernel_timer_start(ctx, max_launches))


def hmc_kernel_timer_read(ctx):
    """(mean ms per launch, launches recorded, kernel name); stops the timer."""
    ms, n = ctypes.c_double(0.0), ctypes.c_int64(0)
    buf = ctypes.create_string_buffer(128)
    _check(lib().hmc_kernel_timer_read(ctx, ctypes.byref(ms), ctypes.byref(n), buf, 128))
    return ms.value, n.value, buf.value.decode()


def hmc_sample_chain_moments(ctx, num_results, num_burnin_steps, adapt: hmc_adapt | None, moments: hmc_moments,
                             trace: hmc_trace | None):
    _check(lib().hmc_sample_chain_moments(ctx, num_results, num_burnin_steps,
                                          ctypes.byref(adapt) if adapt is not None else None, ctypes.byref(moments),
                                          ctypes.byref(trace) if trace is not None else None))


def hmc_set_inverse_temperature(ctx, beta_ptr):
    _check(lib().hmc_set_inverse_temperature(ctx, beta_ptr))


def hmc_remc_swap(ctx, num_replicas: int, swap_index: int, swapped_ptr=None):
    _check(lib().hmc_remc_swap(ctx, num_replicas, swap_index, swapped_ptr))


def hmc_remc_sample_chain(ctx, num_replicas, num_results, num_burnin_steps, adapt: hmc_adapt | None, samples_ptr,
                          trace: hmc_trace | None, swapped_ptr):
    _check(lib().hmc_remc_sample_chain(ctx, num_replicas, num_results, num_burnin_steps,
                                       ctypes.byref(adapt) if adapt is not None else None, samples_ptr,
                                       ctypes.byref(trace) if trace is not None else None, swapped_ptr))


def hmc_get_state(ctx, state_ptr, step_size_ptr) -> int:
    t = ctypes.c_uint64(0)
    _check(lib().hmc_get_state(ctx, state_ptr, step_size_ptr, ctypes.byref(t)))
    return t.value


def hmc_set_state(ctx, state_ptr, step_size_ptr, t: int):
    _check(lib().hmc_set_state(ctx, state_ptr, step_size_ptr, t))


def hmc_destroy(ctx):
    _check(lib().hmc_destroy(ctx))


def hmc_effective_form(ctx) -> int:
    return lib().hmc_effective_form(ctx)


def hmc_autotune(ctx, trial_transitions: int = 3) -> str:
    buf = ctypes.create_string_buffer(4096)
    _check(lib().hmc_autotune(ctx, trial_transitions, buf, len(buf)))
    return buf.value.decode()


def hmc_server_create(hbm_budget_bytes: int, transitions_per_tick: int):
    srv = ctypes.c_void_p()
    _check(lib().hmc_server_create(hbm_budget_bytes, transitions_per_tick, ctypes.byref(srv)))
    return srv


def hmc_server_submit(srv, req: hmc_request) -> int:
    rid = ctypes.c_uint64(0)
    _check(lib().hmc_server_submit(srv, ctypes.byref(req), ctypes.byref(rid)))
    return rid.value


def hmc_server_poll(srv, rid: int):
    state, lat = ctypes.c_int32(0), ctypes.c_double(0)
    _check(lib().hmc_server_poll(srv, rid, ctypes.byref(state), ctypes.byref(lat)))
    return state.value, lat.value


def hmc_server_wait(srv, rid: int):
    state, lat = ctypes.c_int32(0), ctypes.c_double(0)
    _check(lib().hmc_server_wait(srv, rid, ctypes.byref(state), ctypes.byref(lat)))
    return state.value, lat.value


def hmc_server_take(srv, rid: int, dst_ptr):
    _check(lib().hmc_server_take(srv, rid, dst_ptr))


def hmc_server_get_stats(srv) -> dict:
    s = hmc_server_stats()
    _check(lib().hmc_server_get_stats(srv, ctypes.byref(s)))
    return {n: getattr(s, n) for n, _ in hmc_server_stats._fields_}


def hmc_server_destroy(srv):
    _check(lib().hmc_server_destroy(srv))


def hmc_peak_memory(buf, nbytes: int, mode: int, passes: int, reps: int, stream) -> float:
    """GB/s of a streaming read (mode 0, `passes` per launch) or copy (mode 1) over a device buffer."""
    r = ctypes.c_double(0.0)
    _check(lib().hmc_peak_memory(buf, nbytes, mode, passes, reps, stream, ctypes.byref(r)))
    return r.value


def hmc_peak_compute(kind: int, iters: int, reps: int, stream, with_clock: bool = False, waves_per_simd: int = 8):
    """TFLOP/s of one instruction kind (0 FP32 MFMA 16x16x4, 1 FP32 MFMA 4x4x1, 2 BF16 MFMA 16x16x32, 3 FP32 FMA,
    4 BF16 MFMA 32x32x16) at waves_per_simd waves per SIMD;
    with_clock: (TFLOP/s, shader clock in MHz during the last launch)."""
    r, mhz = ctypes.c_double(0.0), ctypes.c_double(0.0)
    _check(lib().hmc_peak_compute(kind, waves_per_simd, iters, reps, stream, ctypes.byref(r), ctypes.byref(mhz)))
    return (r.value, mhz.value) if with_clock else r.value


# ---- convenience wrapper over torch tensors --------------------------------
def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


class Sampler:
    """Owns a context and its workspace.  Target arrays and the initial state
    are torch CUDA tensors; the caller keeps the target arrays alive."""

    def __init__(self, kind, dim, num_chains, num_leapfrog_steps, step_size, init_state, *, prec=None, X=None,
                 y=None, prior_scale=1.0, x_bf16=False, seed=0, state_dtype=None, grad_bf16=False,
                 form=HMC_FORM_AUTO, stream=None):
        import torch
        self.torch = torch
        dev = init_state.device
        f64 = init_state.dtype == torch.float64
        sd = HMC_F64 if f64 else HMC_F32
        if state_dtype is not None:
            sd = state_dtype
        self.keep = [t for t in (prec, X, y, init_state) if t is not None]
        self.target = hmc_target(kind, 0, dim, _ptr(prec), _ptr(X), HMC_BF16 if x_bf16 else HMC_F32, 0,
                                 0 if X is None else X.shape[0], _ptr(y), float(prior_scale))
        self.config = hmc_config(num_chains, num_leapfrog_steps, sd, HMC_BF16 if grad_bf16 else HMC_F32, form,
                                 seed)
        self.dtype = torch.float64 if sd == HMC_F64 else torch.float32
        nbytes = hmc_workspace_size(self.target, self.config)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
        base = self.workspace.data_ptr()
        aligned = (base + 255) & ~255
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        steps = list(step_size) if hasattr(step_size, "__len__") else [step_size]
        self.C, self.D = num_chains, dim
        self.device = dev
        self.ctx = hmc_init(self.target, self.config, _ptr(init_state.contiguous()), steps, ctypes.c_void_p(aligned),
                            nbytes, ctypes.c_void_p(self.stream.cuda_stream))

    @property
    def form(self) -> str:
        return FORM_NAMES.get(hmc_effective_form(self.ctx), "?")

    def autotune(self, trial_transitions: int = 3) -> str:
        return hmc_autotune(self.ctx, trial_transitions)

    def step(self, want_proposal=False):
        torch = self.torch
        C, D = self.C, self.D
        out = dict(is_accepted=torch.empty(C, dtype=torch.uint8, device=self.device),
                   log_accept_ratio=torch.empty(C, dtype=torch.float64, device=self.device),
                   target_log_prob=torch.empty(C, dtype=torch.float64, device=self.device),
                   delta_h=torch.empty(C, dtype=torch.float64, device=self.device))
        if want_proposal:
            out["proposed_state"] = torch.empty(C, D, dtype=self.dtype, device=self.device)
            out["proposed_momentum"] = torch.empty(C, D, dtype=self.dtype, device=self.device)
        so = hmc_step_out(*[_ptr(out.get(k)) for k in ("is_accepted", "log_accept_ratio", "target_log_prob",
                                                         "proposed_state", "proposed_momentum", "delta_h")])
        hmc_step(self.ctx, so)
        return out

    def sample_chain(self, num_results, num_burnin_steps, adapt=False, target_accept=0.8, gamma=0.05, t0=10.0,
                     kappa=0.75, store_samples=True, trace=True, out_samples=None, rate=0.01):
        """out_samples: optional contiguous [R, C, D] device tensor of the state
        dtype that receives the samples (else one is allocated)."""
        torch = self.torch
        C, D, R = self.C, self.D, num_results
        if out_samples is not None:
            if (tuple(out_samples.shape) != (R, C, D) or out_samples.dtype != self.dtype
                    or not out_samples.is_contiguous() or out_samples.device.type != "cuda"):
                raise ValueError("out_samples must be a contiguous [R, C, D] device tensor of the state dtype")
            samples = out_samples
        else:
            samples = torch.empty(R, C, D, dtype=self.dtype, device=self.device) if store_samples else None
        tr = None
        outs = {}
        if trace:
            outs = dict(step_size=torch.empty(R, C, dtype=torch.float64, device=self.device),
                        is_accepted=torch.empty(R, C, dtype=torch.uint8, device=self.device),
                        log_accept_ratio=torch.empty(R, C, dtype=torch.float64, device=self.device),
                        target_log_prob=torch.empty(R, C, dtype=torch.float64, device=self.device))
            tr = hmc_trace(*[_ptr(outs[k]) for k in ("step_size", "is_accepted", "log_accept_ratio",
                                                      "target_log_prob")])
        ad = make_adapt(adapt, target_accept, gamma, t0, kappa, rate)
        hmc_sample_chain(self.ctx, R, num_burnin_steps, ad, _ptr(samples), tr)
        outs["samples"] = samples
        return outs

    def sample_chain_moments(self, num_results, num_burnin_steps, adapt=False, target_accept=0.8, gamma=0.05,
                             t0=10.0, kappa=0.75, rate=0.01, ring_rows=64, batch_len=None, trace=True):
        """Streaming expectations: returns dict(mean [2, C, D], m2 [2, C, D] (FP64,
        per half of the kept draws), batch_sum [R / batch_len, C, D] or None, and the
        traces); no samples are stored."""
        torch = self.torch
        C, D, R = self.C, self.D, num_results
        mean = torch.empty(2, C, D, dtype=torch.float64, device=self.device)
        m2 = torch.empty(2, C, D, dtype=torch.float64, device=self.device)
        bsum = None
        if batch_len:
            bsum = torch.empty(R // batch_len, C, D, dtype=torch.float64, device=self.device)
        ring = torch.empty(max(1, min(ring_rows, max(R, 1))), C, D, dtype=self.dtype, device=self.device)
        outs, tr = {}, None
        if trace:
            outs = dict(step_size=torch.empty(R, C, dtype=torch.float64, device=self.device),
                        is_accepted=torch.empty(R, C, dtype=torch.uint8, device=self.device),
                        log_accept_ratio=torch.empty(R, C, dtype=torch.float64, device=self.device),
                        target_log_prob=torch.empty(R, C, dtype=torch.float64, device=self.device))
            tr = hmc_trace(*[_ptr(outs[k]) for k in ("step_size", "is_accepted", "log_accept_ratio",
                                                      "target_log_prob")])
        mo = hmc_moments(_ptr(mean).value, _ptr(m2).value, None if bsum is None else _ptr(bsum).value,
                         int(batch_len or 0), _ptr(ring).value, ring.shape[0])
        ad = make_adapt(adapt, target_accept, gamma, t0, kappa, rate)
        hmc_sample_chain_moments(self.ctx, R, num_burnin_steps, ad, mo, tr)
        outs.update(mean=mean, m2=m2, batch_sum=bsum, ring=ring)
        return outs

    def nuts_sample_chain(self, num_results, num_burnin_steps, max_depth=10, store_samples=True, adapt=False,
                          target_accept=0.8, gamma=0.05, t0=10.0, kappa=0.75, rate=0.01):
        """No-U-Turn sampler from the current state with each chain's step size,
        adapted during burn-in when adapt is set (as sample_chain's).  Returns
        dict(samples [R, C, D] or None, tree_depth [R, C], n_leapfrog [R, C],
        accept_stat [R, C])."""
        torch = self.torch
        C, D, R = self.C, self.D, num_results
        nb = ctypes.c_size_t(0)
        _check(lib().hmc_nuts_workspace_size(self.ctx, max_depth, ctypes.byref(nb)))
        ws = torch.empty(max(int(nb.value), 1), dtype=torch.uint8, device=self.device)
        samples = torch.empty(R, C, D, dtype=self.dtype, device=self.device) if store_samples else None
        depth = torch.empty(R, C, dtype=torch.int32, device=self.device)
        nleap = torch.empty(R, C, dtype=torch.int32, device=self.device)
        stat = torch.empty(R, C, dtype=torch.float64, device=self.device)
        ad = make_adapt(adapt, target_accept, gamma, t0, kappa, rate)
        _check(lib().hmc_nuts_sample_chain(self.ctx, max_depth, R, num_burnin_steps, ctypes.byref(ad) if ad else None,
                                           _ptr(ws), nb.value, _ptr(samples), _ptr(depth), _ptr(nleap), _ptr(stat)))
        return dict(samples=samples, tree_depth=depth, n_leapfrog=nleap, accept_stat=stat)

    def set_transform_scale(self, scale):
        """Diagonal affine bijector x = shift + scale * z (the shift does not enter
        the dynamics): scale [D] (any array-like), or None for the identity."""
        if scale is None:
            _check(lib().hmc_set_transform_scale(self.ctx, None))
            return
        sc = self.torch.as_tensor(scale, dtype=self.torch.float64).to(self.device).contiguous()
        self.keep.append(sc)
        _check(lib().hmc_set_transform_scale(self.ctx, _ptr(sc)))

    def set_inverse_temperature(self, beta):
        """beta: [C] FP64 device tensor (one value per chain), or None for 1."""
        if beta is None:
            hmc_set_inverse_temperature(self.ctx, None)
            return
        beta = beta.to(device=self.device, dtype=self.torch.float64).contiguous()
        self.keep.append(beta)
        hmc_set_inverse_temperature(self.ctx, _ptr(beta))

    def remc_swap(self, num_replicas, swap_index, swapped=True):
        torch = self.torch
        sw = torch.empty(self.C, dtype=torch.uint8, device=self.device) if swapped else None
        hmc_remc_swap(self.ctx, num_replicas, swap_index, _ptr(sw))
        return sw

    def remc_sample_chain(self, num_replicas, num_results, num_burnin_steps, adapt=False, target_accept=0.8,
                          gamma=0.05, t0=10.0, kappa=0.75, store_samples=True, trace=True, swapped=True,
                          rate=0.01):
        """Replica exchange: chains are num_replicas blocks of C / num_replicas
        (replica-major); returns samples (after each exchange), traces and the
        exchange flags [R, C]."""
        torch = self.torch
        C, D, R = self.C, self.D, num_results
        samples = torch.empty(R, C, D, dtype=self.dtype, device=self.device) if store_samples else None
        outs, tr = {}, None
        if trace:
            outs = dict(step_size=torch.empty(R, C, dtype=torch.float64, device=self.device),
                        is_accepted=torch.empty(R, C, dtype=torch.uint8, device=self.device),
                        log_accept_ratio=torch.empty(R, C, dtype=torch.float64, device=self.device),
                        target_log_prob=torch.empty(R, C, dtype=torch.float64, device=self.device))
            tr = hmc_trace(*[_ptr(outs[k]) for k in ("step_size", "is_accepted", "log_accept_ratio",
                                                      "target_log_prob")])
        sw = torch.empty(R, C, dtype=torch.uint8, device=self.device) if swapped else None
        ad = make_adapt(adapt, target_accept, gamma, t0, kappa, rate)
        hmc_remc_sample_chain(self.ctx, num_replicas, R, num_burnin_steps, ad, _ptr(samples), tr, _ptr(sw))
        outs["samples"] = samples
        outs["swapped"] = sw
        return outs

    def get_state(self):
        torch = self.torch
        x = torch.empty(self.C, self.D, dtype=self.dtype, device=self.device)
        e = torch.empty(self.C, dtype=torch.float64, device=self.device)
        t = hmc_get_state(self.ctx, _ptr(x), _ptr(e))
        return x, e, t

    def set_state(self, x, eps=None, t=0):
        self.keep.append(x)
        hmc_set_state(self.ctx, _ptr(x.contiguous()), _ptr(eps), t)

    def close(self):
        if self.ctx is not None:
            hmc_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def sampler_for(w, device="cuda", form=HMC_FORM_AUTO, grad_bf16=False, num_chains=None, seed=None, x0=None,
                step_size=None):
    """Build a Sampler for a workloads.Workload (inputs copied to the device)."""
    import numpy as np
    import torch
    dev = torch.device(device)
    C = w.num_chains if num_chains is None else num_chains
    x0 = w.x0[:C] if x0 is None else x0
    init = torch.from_numpy(np.ascontiguousarray(x0)).to(dev)
    prec = X = y = None
    x_bf16 = False
    if w.prec is not None:
        prec = torch.from_numpy(np.ascontiguousarray(w.prec)).to(dev)
    if w.X is not None:
        if w.X_bf16 is not None:
            X = torch.from_numpy(w.X_bf16.view(np.int16)).to(dev)
            x_bf16 = True
        else:
            X = torch.from_numpy(np.ascontiguousarray(w.X)).to(dev)
        y = torch.from_numpy(w.y).to(dev)
    eps = w.step_size if step_size is None else step_size
    s = Sampler(w.kind, w.dim, C, w.num_leapfrog_steps, eps, init, prec=prec, X=X, y=y,
                prior_scale=w.prior_scale, x_bf16=x_bf16, seed=w.seed if seed is None else seed, form=form,
                grad_bf16=grad_bf16)
    return s


class Server:
    """Continuous-batching sampling server over torch tensors.  submit() keeps
    references to every tensor of a request until it is collected."""

    def __init__(self, hbm_budget_bytes: int, transitions_per_tick: int = 10, device="cuda"):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.srv = hmc_server_create(hbm_budget_bytes, transitions_per_tick)
        self.keep = {}

    def submit(self, w, **kw):
        """Queue a workloads.Workload as one sampling request; returns its id."""
        return self.submit_prepared(self.prepare(w, **kw))

    def submit_prepared(self, prep):
        req, keep = prep
        rid = hmc_server_submit(self.srv, req)
        self.keep[rid] = keep
        return rid

    def prepare(self, w, num_chains=None, seed=None, form=HMC_FORM_AUTO, grad_bf16=False, server_samples=False,
                trace=True):
        """Upload a request's inputs and allocate its outputs; submit_prepared queues it."""
        import numpy as np
        torch = self.torch
        dev = self.device
        C = w.num_chains if num_chains is None else num_chains
        init = torch.from_numpy(np.ascontiguousarray(w.x0[:C])).to(dev)
        prec = X = y = None
        x_bf16 = False
        if w.prec is not None:
            prec = torch.from_numpy(np.ascontiguousarray(w.prec)).to(dev)
        if w.X is not None:
            if w.X_bf16 is not None:
                X = torch.from_numpy(w.X_bf16.view(np.int16)).to(dev)
                x_bf16 = True
            else:
                X = torch.from_numpy(np.ascontiguousarray(w.X)).to(dev)
            y = torch.from_numpy(w.y).to(dev)
        dt = torch.float64 if w.state_dtype == "f64" else torch.float32
        R = w.num_results
        samples = None if server_samples else torch.empty(R, C, w.dim, dtype=dt, device=dev)
        outs = {}
        tr = hmc_trace()
        if trace:
            outs = dict(step_size=torch.empty(R, C, dtype=torch.float64, device=dev),
                        is_accepted=torch.empty(R, C, dtype=torch.uint8, device=dev),
                        log_accept_ratio=torch.empty(R, C, dtype=torch.float64, device=dev),
                        target_log_prob=torch.empty(R, C, dtype=torch.float64, device=dev))
            tr = hmc_trace(*[_ptr(outs[k]) for k in ("step_size", "is_accepted", "log_accept_ratio",
                                                      "target_log_prob")])
        target = hmc_target(w.kind, 0, w.dim, _ptr(prec), _ptr(X), HMC_BF16 if x_bf16 else HMC_F32, 0,
                            0 if X is None else X.shape[0], _ptr(y), float(w.prior_scale))
        config = hmc_config(C, w.num_leapfrog_steps, HMC_F64 if w.state_dtype == "f64" else HMC_F32,
                            HMC_BF16 if grad_bf16 else HMC_F32, form, w.seed if seed is None else seed)
        adapt = hmc_adapt(1 if w.adapt else 0, HMC_ADAPT_DUAL_AVERAGING, 0.8, 0.05, 10.0, 0.75, 0.01)
        torch.cuda.synchronize(dev)    # inputs are on the device before the worker reads them
        req = hmc_request(target, config, _ptr(init), float(w.step_size), R, w.num_burnin, adapt, _ptr(samples), tr)
        outs["samples"] = samples
        keep = dict(tensors=[t for t in (init, prec, X, y) if t is not None], outs=outs, shape=(R, C, w.dim),
                    dtype=dt)
        return req, keep

    def poll(self, rid):
        return hmc_server_poll(self.srv, rid)

    def wait(self, rid):
        """Block until done; returns (outputs dict, latency seconds)."""
        state, lat = hmc_server_wait(self.srv, rid)
        k = self.keep[rid]
        out = k["outs"]
        if out.get("samples") is None and k["shape"][0] > 0:
            dst = self.torch.empty(*k["shape"], dtype=k["dtype"], device=self.device)
            hmc_server_take(self.srv, rid, _ptr(dst))
            out["samples"] = dst
        return out, lat

    def stats(self):
        return hmc_server_get_stats(self.srv)

    def close(self):
        if self.srv is not None:
            hmc_server_destroy(self.srv)
            self.srv = None
