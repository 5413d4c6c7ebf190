"""Python binding of libppp, the MI355X implementation of the parallel pulling
protocol (V. A. Ngo, arXiv:1105.4840, Sec. III(ii)).

Argument marshalling only: every step of the protocol runs in the library's
HIP kernels.  PyTorch provides device memory (workspace tensors) and the
stream; results come back as numpy arrays.  Functions keep the C names
(``ppp_create``, ``ppp_run``, ...); ``run()`` is the one-call convenience.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libppp.so")

PPP_OK, PPP_E_INVALID_ARG, PPP_E_OUT_OF_MEMORY, PPP_E_DEVICE, PPP_E_NUMERICAL, PPP_E_STATE, PPP_E_UNSUPPORTED = range(7)
PPP_FLAG_SEQUENTIAL = 1
PPP_FLAG_FREE_ENSEMBLE = 2
# entries of the turn-on array (include/ppp.h, PPP_ON_*)
TURN_ON_FIELDS = ["eq5_first", "eq5_first_se", "eq6_first", "eq6_first_se", "lower_first", "upper_first",
                  "eq5_last", "eq5_last_se", "eq6_last", "eq6_last_se", "lower_last", "upper_last",
                  "eq10_log", "eq10_log_se", "free_n", "free_blown", "free_mean", "free_std", "free_under",
                  "free_over"]
PPP_MLP_HIDDEN = 64
PPP_MLP_PARAMS = 64 + 64 + 64 * 64 + 64 + 64 + 1

_dp = ctypes.POINTER(ctypes.c_double)
_fp = ctypes.POINTER(ctypes.c_float)
_i64p = ctypes.POINTER(ctypes.c_int64)
_u64p = ctypes.POINTER(ctypes.c_uint64)
_i32p = ctypes.POINTER(ctypes.c_int32)


class PppError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} (status {status})")
        self.status = status


class ppp_pot1d(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("a", ctypes.c_double), ("b", ctypes.c_double),
                ("kappa", ctypes.c_double), ("mobility", ctypes.c_double)]


class ppp_chain(ctypes.Structure):
    _fields_ = [("n_beads", ctypes.c_int32), ("k_bond", ctypes.c_double), ("r0", ctypes.c_double),
                ("k_angle", ctypes.c_double), ("lj_eps", ctypes.c_double), ("lj_sigma", ctypes.c_double),
                ("lj_rc", ctypes.c_double), ("rc_mode", ctypes.c_int32), ("mass", ctypes.c_double),
                ("gamma", ctypes.c_double)]


class ppp_problem(ctypes.Structure):
    _fields_ = [("model", ctypes.c_int32), ("pot1d", ppp_pot1d), ("chain", ppp_chain),
                ("n_windows", ctypes.c_int32), ("lambda_", _dp),
                ("k", ctypes.c_double), ("kT", ctypes.c_double), ("dt", ctypes.c_double),
                ("n_steps", ctypes.c_int64), ("n_equil", ctypes.c_int64), ("n_pull", ctypes.c_int64),
                ("sample_every", ctypes.c_int32), ("n_replicas", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("precision", ctypes.c_int32), ("integrator_1d", ctypes.c_int32), ("init_coords", _dp),
                ("xi_min", ctypes.c_double), ("xi_bin", ctypes.c_double), ("xi_nbins", ctypes.c_int32),
                ("w_bin", ctypes.c_double), ("w_half_bins", ctypes.c_int32), ("n_jack_blocks", ctypes.c_int32),
                ("xi_bound", ctypes.c_double), ("flags", ctypes.c_uint32)]


_RESULT_S = ["dF_je", "dF_je_se", "dF_fluct", "dF_fluct_se", "dF_gauss", "dF_gauss_se", "dF_com", "dF_com_se",
             "dF_unc", "dF_rev", "dF_je_hist", "dF_je_hist_mid", "dF_je_var_paper", "sigma_w"]
_RESULT_S_I64 = ["q_bins"]
_RESULT_S2 = ["work_lost", "xi_mean", "xi_std", "gamma2", "xi_min_sample", "xi_max_sample", "lse_fwd", "lse_rev"]
_RESULT_S_I64_2 = ["n_samples", "n_blown_up"]
_RESULT_P = ["kish_frac", "overlap_ovl", "dlambda_over_sigma", "dlambda_over_reach"]
_RESULT_LIT = ["dF_fluct_literal", "dF_gauss_literal", "dF_je_hist_literal"]
_RESULT_REV = ["dF_rev_hist", "crooks_ovl", "dF_crooks"]
_RESULT_LSQ = ["sigma_lsq", "gamma2_lsq", "dF_gauss_lsq"]


class ppp_result(ctypes.Structure):
    _fields_ = ([(n, _dp) for n in _RESULT_S] + [(n, _i64p) for n in _RESULT_S_I64] +
                [(n, _dp) for n in _RESULT_S2] + [(n, _i64p) for n in _RESULT_S_I64_2] +
                [(n, _dp) for n in _RESULT_P] + [("criterion_ok", _i32p)] + [(n, _dp) for n in _RESULT_LIT] +
                [("xi_hist", _u64p), ("xi_under_over", _u64p), ("work_hist", _dp)] +
                [("turn_on", _dp), ("G", _dp), ("G_se", _dp), ("xi_hist_free", _u64p)] +
                [(n, _dp) for n in _RESULT_REV] + [("work_hist_rev", _dp)] + [(n, _dp) for n in _RESULT_LSQ])


class ppp_timings(ctypes.Structure):
    _fields_ = [("sim_ms", ctypes.c_double), ("reduce_ms", ctypes.c_double), ("appc_ms", ctypes.c_double),
                ("total_ms", ctypes.c_double), ("replica_steps", ctypes.c_int64), ("sim_launches", ctypes.c_int32),
                ("variant_lanes", ctypes.c_int32), ("variant_beads_per_lane", ctypes.c_int32),
                ("last_advance_ms", ctypes.c_double)]


class ppp_adaptive(ctypes.Structure):
    _fields_ = [("budget_replica_steps", ctypes.c_int64), ("initial_windows", ctypes.c_int32),
                ("max_rounds", ctypes.c_int32), ("max_windows", ctypes.c_int32),
                ("target_dl_over_sigma", ctypes.c_double), ("train_iters", ctypes.c_int32),
                ("lr", ctypes.c_double), ("init_seed", ctypes.c_uint64), ("explore_replicas", ctypes.c_int32),
                ("explore_steps", ctypes.c_int64), ("min_production_steps", ctypes.c_int64),
                ("placement", ctypes.c_int32)]

PPP_PLACE_LEARNED, PPP_PLACE_EXPLORED = 0, 1
PPP_STATIC_WORKSPACE_BYTES = 64 << 20          # include/ppp.h
PPP_PROBE_SGPR_OPERANDS, PPP_PROBE_VGPR_OPERANDS = 0, 1   # include/ppp_probe.h


_lib = None


def lib():
    """Loads libppp.so; raises if it is not built (there is no CPU fallback)."""
    global _lib
    if _lib is None:
        # torch ships its own HIP runtime under the same soname; loading torch first makes
        # libppp bind to that one, so the process holds a single HIP runtime
        import torch  # noqa: F401
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"libppp.so not found at {LIB_PATH}: build it with __graft_entry__.build() "
                              "(python paper_1105_4840_amd/build.py)")
        L = ctypes.CDLL(LIB_PATH)
        H = ctypes.c_void_p
        vp = ctypes.c_void_p
        st = ctypes.c_int
        sig = {
            "ppp_create": ([ctypes.POINTER(ppp_problem), ctypes.POINTER(H)], st),
            "ppp_batch_create": ([ctypes.POINTER(ppp_problem), ctypes.c_int32, ctypes.c_char_p, ctypes.POINTER(H)], st),
            "ppp_workspace_size": ([H, ctypes.POINTER(ctypes.c_size_t)], st),
            "ppp_run": ([H, vp, ctypes.c_size_t, vp], st),
            "ppp_run_static": ([H, vp], st),
            "ppp_begin": ([H, vp, ctypes.c_size_t, vp], st),
            "ppp_advance": ([H, ctypes.c_int64, vp], st),
            "ppp_finalize": ([H, vp], st),
            "ppp_steps_done": ([H, _i64p], st),
            "ppp_get_result": ([H, ctypes.POINTER(ppp_result)], st),
            "ppp_batch_get_result": ([H, ctypes.c_int32, ctypes.POINTER(ppp_result)], st),
            "ppp_get_timings": ([H, ctypes.POINTER(ppp_timings)], st),
            "ppp_checkpoint": ([H, vp, ctypes.POINTER(ctypes.c_size_t)], st),
            "ppp_restore": ([H, vp, ctypes.c_size_t, vp, ctypes.c_size_t, vp], st),
            "ppp_destroy": ([H], st),
            "ppp_status_string": ([st], ctypes.c_char_p),
            "ppp_last_error": ([H], ctypes.c_char_p),
            "ppp_create_error": ([], ctypes.c_char_p),
            "ppp_eval_forces": ([H, vp, ctypes.c_size_t, vp, ctypes.c_int32, ctypes.c_double, vp, vp, vp], st),
            "ppp_trajectory": ([H, vp, ctypes.c_size_t, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, vp, vp], st),
            "ppp_philox": ([ctypes.c_uint64] + [ctypes.c_uint32] * 4 + [ctypes.c_int32, vp, vp, vp, vp, vp, vp], st),
            "ppp_probe_valu": ([ctypes.c_int32, ctypes.c_int32, ctypes.c_float, ctypes.c_float, ctypes.c_int32, vp, vp],
                               st),
            "ppp_mlp_forward": ([vp, vp, ctypes.c_int32, vp, vp, vp], st),
            "ppp_mlp_grad": ([vp, vp, vp, vp, vp, vp, ctypes.c_int32, vp, vp, vp], st),
            "ppp_mlp_adam": ([vp, vp, vp, vp, ctypes.c_float, ctypes.c_int32, vp], st),
            "ppp_adaptive_workspace_size": ([ctypes.POINTER(ppp_problem), ctypes.POINTER(ppp_adaptive),
                                             ctypes.POINTER(ctypes.c_size_t)], st),
            "ppp_adaptive_run": ([ctypes.POINTER(ppp_problem), ctypes.POINTER(ppp_adaptive), vp, ctypes.c_size_t, vp,
                                  _dp, _i32p, _i64p, ctypes.POINTER(ppp_result)], st),
            "ppp_autotune": ([ctypes.c_char_p, vp, ctypes.c_size_t, vp], st),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


EXPORTED = ["ppp_create", "ppp_batch_create", "ppp_workspace_size", "ppp_run", "ppp_run_static", "ppp_begin",
            "ppp_advance",
            "ppp_finalize", "ppp_steps_done", "ppp_get_result", "ppp_batch_get_result", "ppp_get_timings",
            "ppp_checkpoint", "ppp_restore", "ppp_destroy", "ppp_status_string", "ppp_last_error",
            "ppp_create_error", "ppp_eval_forces", "ppp_trajectory", "ppp_philox", "ppp_probe_valu", "ppp_mlp_forward",
            "ppp_mlp_grad", "ppp_mlp_adam", "ppp_adaptive_workspace_size", "ppp_adaptive_run", "ppp_autotune"]


def _check(status, handle=None, where=""):
    if status != PPP_OK and status != PPP_E_NUMERICAL:
        L = lib()
        msg = L.ppp_last_error(handle).decode() if handle else L.ppp_create_error().decode()
        raise PppError(status, f"{where}: {L.ppp_status_string(status).decode()}: {msg}")
    return status


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


# ----------------------------------------------------------------------------- problems

def make_problem(prob: dict):
    """Builds the ppp_problem struct for a problem dict (keys as in ppp_inputs);
    returns (struct, keepalive)."""
    lam = np.ascontiguousarray(np.asarray(prob["lambda"], dtype=np.float64))
    ic = prob.get("init_coords")
    init = None if ic is None else np.ascontiguousarray(np.asarray(ic, dtype=np.float64).ravel())
    chain = prob["model"] == "chain"
    p = ppp_problem()
    p.model = 1 if chain else 0
    p.pot1d = ppp_pot1d(int(prob.get("pot_kind", 0)), float(prob.get("pot_a", 5.0)), float(prob.get("pot_b", 1.0)),
                        float(prob.get("pot_kappa", 0.0)), float(prob.get("mobility", 1.0)))
    p.chain = ppp_chain(int(prob.get("n_beads", 2)), float(prob.get("k_bond", 100.0)), float(prob.get("r0", 1.0)),
                        float(prob.get("k_angle", 5.0)), float(prob.get("lj_eps", 1.0)),
                        float(prob.get("lj_sigma", 1.0)), float(prob.get("lj_rc", 2.5)),
                        int(prob.get("rc_mode", 0)), float(prob.get("mass", 1.0)), float(prob.get("gamma", 1.0)))
    p.n_windows = len(lam)
    p.lambda_ = lam.ctypes.data_as(_dp)
    p.k = float(prob["k"]); p.kT = float(prob["kT"]); p.dt = float(prob["dt"])
    p.n_steps = int(prob["n_steps"]); p.n_equil = int(prob["n_equil"]); p.n_pull = int(prob.get("n_pull", 0))
    p.sample_every = int(prob["sample_every"]); p.n_replicas = int(prob["n_replicas"])
    p.seed = int(prob["seed"])
    p.precision = 1 if prob.get("precision", "fp32") == "fp64" else 0
    p.integrator_1d = int(prob.get("integrator_1d", 0))
    p.init_coords = None if init is None else init.ctypes.data_as(_dp)
    p.xi_min = float(prob["xi_min"]); p.xi_bin = float(prob["xi_bin"]); p.xi_nbins = int(prob["xi_nbins"])
    p.w_bin = float(prob.get("w_bin", 0.01)); p.w_half_bins = int(prob.get("w_half_bins", 0))
    p.n_jack_blocks = int(prob.get("n_blocks", 0)); p.xi_bound = float(prob.get("xi_bound", 1.0e4))
    p.flags = (int(prob.get("flags", 0)) | (PPP_FLAG_SEQUENTIAL if prob.get("sequential", False) else 0) |
               (PPP_FLAG_FREE_ENSEMBLE if prob.get("free_ensemble", False) else 0))
    return p, (lam, init)


def ppp_create(prob: dict):
    p, keep = make_problem(prob)
    h = ctypes.c_void_p()
    _check(lib().ppp_create(ctypes.byref(p), ctypes.byref(h)), None, "ppp_create")
    return h


def ppp_batch_create(probs, tune_table_path=None):
    arr = (ppp_problem * len(probs))()
    keep = []
    for i, pr in enumerate(probs):
        p, k = make_problem(pr)
        arr[i] = p
        keep.append(k)
    h = ctypes.c_void_p()
    path = None if tune_table_path is None else str(tune_table_path).encode()
    _check(lib().ppp_batch_create(arr, len(probs), path, ctypes.byref(h)), None, "ppp_batch_create")
    return h


def ppp_workspace_size(h) -> int:
    n = ctypes.c_size_t()
    _check(lib().ppp_workspace_size(h, ctypes.byref(n)), h, "ppp_workspace_size")
    return int(n.value)


def workspace(h, device="cuda"):
    """A device workspace tensor of ppp_workspace_size bytes (256-byte aligned by the allocator)."""
    import torch
    n = ppp_workspace_size(h)
    return torch.empty(max(n, 256), dtype=torch.uint8, device=device)


def ppp_run(h, ws, stream=None):
    return _check(lib().ppp_run(h, _ptr(ws), ws.numel(), _stream(stream)), h, "ppp_run")


def ppp_run_static(h, stream=None):
    return _check(lib().ppp_run_static(h, _stream(stream)), h, "ppp_run_static")


def ppp_begin(h, ws, stream=None):
    return _check(lib().ppp_begin(h, _ptr(ws), ws.numel(), _stream(stream)), h, "ppp_begin")


def ppp_advance(h, n_steps, stream=None):
    return _check(lib().ppp_advance(h, int(n_steps), _stream(stream)), h, "ppp_advance")


def ppp_finalize(h, stream=None):
    return _check(lib().ppp_finalize(h, _stream(stream)), h, "ppp_finalize")


def ppp_steps_done(h) -> int:
    n = ctypes.c_int64()
    _check(lib().ppp_steps_done(h, ctypes.byref(n)), h, "ppp_steps_done")
    return int(n.value)


def _result_buffers(prob):
    s = len(prob["lambda"]); K = int(prob["xi_nbins"]); M = int(prob.get("w_half_bins", 0))
    bufs = {}
    r = ppp_result()
    for n in _RESULT_S + _RESULT_S2 + _RESULT_LIT:
        bufs[n] = np.full(s, np.nan); setattr(r, n, bufs[n].ctypes.data_as(_dp))
    for n in _RESULT_S_I64 + _RESULT_S_I64_2:
        bufs[n] = np.zeros(s, dtype=np.int64); setattr(r, n, bufs[n].ctypes.data_as(_i64p))
    for n in _RESULT_P:
        bufs[n] = np.full(s - 1, np.nan); setattr(r, n, bufs[n].ctypes.data_as(_dp))
    bufs["criterion_ok"] = np.zeros(s - 1, dtype=np.int32); r.criterion_ok = bufs["criterion_ok"].ctypes.data_as(_i32p)
    bufs["xi_hist"] = np.zeros((s, K), dtype=np.uint64); r.xi_hist = bufs["xi_hist"].ctypes.data_as(_u64p)
    bufs["xi_under_over"] = np.zeros((s, 2), dtype=np.uint64); r.xi_under_over = bufs["xi_under_over"].ctypes.data_as(_u64p)
    for n in _RESULT_REV + _RESULT_LSQ:
        bufs[n] = np.full(s, np.nan); setattr(r, n, bufs[n].ctypes.data_as(_dp))
    if M > 0:
        bufs["work_hist"] = np.zeros((s, 2 * M + 1)); r.work_hist = bufs["work_hist"].ctypes.data_as(_dp)
        bufs["work_hist_rev"] = np.zeros((s, 2 * M + 1)); r.work_hist_rev = bufs["work_hist_rev"].ctypes.data_as(_dp)
    else:
        r.work_hist = None
        r.work_hist_rev = None
    bufs["turn_on_raw"] = np.full(len(TURN_ON_FIELDS), np.nan); r.turn_on = bufs["turn_on_raw"].ctypes.data_as(_dp)
    for n in ("G", "G_se"):
        bufs[n] = np.full(s, np.nan); setattr(r, n, bufs[n].ctypes.data_as(_dp))
    bufs["xi_hist_free"] = np.zeros(K, dtype=np.uint64); r.xi_hist_free = bufs["xi_hist_free"].ctypes.data_as(_u64p)
    return r, bufs


def ppp_get_result(h, prob, index=None):
    """Results as a dict of numpy arrays; 'status' is PPP_OK or PPP_E_NUMERICAL."""
    r, bufs = _result_buffers(prob)
    if index is None:
        st = _check(lib().ppp_get_result(h, ctypes.byref(r)), h, "ppp_get_result")
    else:
        st = _check(lib().ppp_batch_get_result(h, int(index), ctypes.byref(r)), h, "ppp_batch_get_result")
    bufs["status"] = st
    bufs["turn_on"] = dict(zip(TURN_ON_FIELDS, (float(v) for v in bufs.pop("turn_on_raw"))))
    return bufs


def ppp_batch_get_result(h, prob, index):
    return ppp_get_result(h, prob, index)


def ppp_get_timings(h) -> dict:
    t = ppp_timings()
    _check(lib().ppp_get_timings(h, ctypes.byref(t)), h, "ppp_get_timings")
    return {n: getattr(t, n) for n, _ in ppp_timings._fields_}


def ppp_checkpoint(h) -> bytes:
    n = ctypes.c_size_t()
    _check(lib().ppp_checkpoint(h, None, ctypes.byref(n)), h, "ppp_checkpoint")
    buf = ctypes.create_string_buffer(n.value)
    _check(lib().ppp_checkpoint(h, buf, ctypes.byref(n)), h, "ppp_checkpoint")
    return buf.raw


def ppp_restore(h, ws, blob: bytes, stream=None):
    buf = ctypes.create_string_buffer(blob, len(blob))
    return _check(lib().ppp_restore(h, _ptr(ws), ws.numel(), buf, len(blob), _stream(stream)), h, "ppp_restore")


def ppp_destroy(h):
    if h:
        lib().ppp_destroy(h)


def ppp_eval_forces(h, ws, coords, lam, stream=None):
    """coords: device fp64 tensor [n, dof]; returns (forces [n, dof], energy [n, 5]) device tensors."""
    import torch
    coords = coords.contiguous()
    n = coords.shape[0]
    f = torch.empty_like(coords)
    e = torch.empty((n, 5), dtype=torch.float64, device=coords.device)
    _check(lib().ppp_eval_forces(h, _ptr(ws), ws.numel(), _ptr(coords), n, float(lam), _ptr(f), _ptr(e),
                                 _stream(stream)), h, "ppp_eval_forces")
    return f, e


def ppp_trajectory(h, ws, window, replica, n_steps, dof, stream=None):
    import torch
    out = torch.full((n_steps + 1, dof), float("nan"), dtype=torch.float64, device=ws.device)
    _check(lib().ppp_trajectory(h, _ptr(ws), ws.numel(), int(window), int(replica), int(n_steps), _ptr(out),
                                _stream(stream)), h, "ppp_trajectory")
    return out


def ppp_philox(seed, c0, c1, c2, c3, n, device="cuda", stream=None):
    """(words u32 [n,4], fp64 normals [n,4], fp32 normals [n,4], fp64 normals [n,6], fp32 normals [n,6])
    for counters (c0+i, c1, c2, c3): the 1-D model's four normals per block and the chain's six."""
    import torch
    words = torch.zeros((n, 4), dtype=torch.int32, device=device)
    z64 = torch.zeros((n, 4), dtype=torch.float64, device=device)
    z32 = torch.zeros((n, 4), dtype=torch.float32, device=device)
    y64 = torch.zeros((n, 6), dtype=torch.float64, device=device)
    y32 = torch.zeros((n, 6), dtype=torch.float32, device=device)
    st = lib().ppp_philox(int(seed), c0, c1, c2, c3, int(n), _ptr(words), _ptr(z64), _ptr(z32), _ptr(y64), _ptr(y32),
                          _stream(stream))
    _check(st, None, "ppp_philox")
    return (words.cpu().numpy().view(np.uint32), z64.cpu().numpy(), z32.cpu().numpy(), y64.cpu().numpy(),
            y32.cpu().numpy())


def ppp_probe_valu(n_blocks, iters, b=0.999999, c=1e-7, out=None, device="cuda", stream=None, vgpr_operands=False):
    """Launches the fp32 FMA issue-rate probe (16 * iters flops per thread, n_blocks x 256
    threads) on `stream` and returns its device output (one fp32 per thread); b and c in
    scalar registers, or in vector registers with vgpr_operands."""
    import torch
    n = int(n_blocks) * 256
    if out is None:
        out = torch.empty(n, dtype=torch.float32, device=device)
    if out.numel() < n or out.dtype != torch.float32:
        raise ValueError("ppp_probe_valu: out must hold n_blocks * 256 fp32 values")
    mode = PPP_PROBE_VGPR_OPERANDS if vgpr_operands else PPP_PROBE_SGPR_OPERANDS
    _check(lib().ppp_probe_valu(int(n_blocks), int(iters), float(b), float(c), mode, _ptr(out), _stream(stream)),
           None, "ppp_probe_valu")
    return out


def ppp_adaptive_run(base: dict, adaptive: dict, stream=None, device="cuda"):
    """Adaptive protocol with learned window placement; returns (results dict on the
    production windows, lambda array, replica-steps used)."""
    import torch
    p, keep = make_problem(base)
    a = ppp_adaptive(int(adaptive["budget_replica_steps"]), int(adaptive.get("initial_windows", 11)),
                     int(adaptive.get("max_rounds", 4)), int(adaptive.get("max_windows", 256)),
                     float(adaptive.get("target_dl_over_sigma", 1.0)), int(adaptive.get("train_iters", 400)),
                     float(adaptive.get("lr", 3e-3)), int(adaptive.get("init_seed", 1)),
                     int(adaptive.get("explore_replicas", 0)), int(adaptive.get("explore_steps", 0)),
                     int(adaptive.get("min_production_steps", 0)),
                     {"learned": PPP_PLACE_LEARNED, "explored": PPP_PLACE_EXPLORED}[adaptive.get("placement", "learned")])
    n = ctypes.c_size_t()
    _check(lib().ppp_adaptive_workspace_size(ctypes.byref(p), ctypes.byref(a), ctypes.byref(n)), None,
           "ppp_adaptive_workspace_size")
    ws = torch.empty(max(int(n.value), 256), dtype=torch.uint8, device=device)
    smax = int(a.max_windows)
    shaped = dict(base, **{"lambda": np.zeros(smax)})
    r, bufs = _result_buffers(shaped)
    lam = np.zeros(smax)
    nw = ctypes.c_int32()
    used = ctypes.c_int64()
    st = lib().ppp_adaptive_run(ctypes.byref(p), ctypes.byref(a), _ptr(ws), ws.numel(), _stream(stream),
                                lam.ctypes.data_as(_dp), ctypes.byref(nw), ctypes.byref(used), ctypes.byref(r))
    _check(st, None, "ppp_adaptive_run")
    s = int(nw.value)
    out = {}
    for key, v in bufs.items():
        if isinstance(v, np.ndarray) and v.ndim >= 1 and v.shape[0] in (smax, smax - 1):
            out[key] = v[:s] if v.shape[0] == smax else v[:s - 1]
        else:
            out[key] = v
    out["status"] = st
    return out, lam[:s], int(used.value)


def run(prob: dict, stream=None, device="cuda"):
    """Creates, runs and destroys a handle; returns (results dict, timings dict)."""
    import torch
    h = ppp_create(prob)
    try:
        ws = workspace(h, device)
        ppp_run(h, ws, stream)
        res = ppp_get_result(h, prob)
        tim = ppp_get_timings(h)
        torch.cuda.synchronize()
        del ws
        return res, tim
    finally:
        ppp_destroy(h)
