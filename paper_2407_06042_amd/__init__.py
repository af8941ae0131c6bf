"""Python binding of libdmala.so, the MI355X DMALA MIMO detector.

Argument marshalling only: every step of detection runs in the library's HIP
kernels.  PyTorch supplies device memory and the current HIP stream.  The
library is loaded from this directory; if it is missing or fails to load, every
entry point raises -- there is no CPU fallback.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdmala.so")

FP64, FP32, BF16, FP16 = 0, 1, 2, 3
PRECOND, NAIVE, LEARNED, MHGD = 0, 1, 2, 3
PRECISIONS = {"fp64": FP64, "fp32": FP32, "bf16": BF16, "fp16": FP16}
PROPOSALS = {"precond": PRECOND, "naive": NAIVE, "learned": LEARNED, "mhgd": MHGD}
MLP_PARAMS = 4932     # DMALA_MLP_PARAMS
TRAIN_ROW = 12        # DMALA_TRAIN_ROW
STATIC_SCRATCH_BYTES = 64 << 20   # DMALA_STATIC_SCRATCH_BYTES
STATUS = {0: "DMALA_OK", -1: "DMALA_ERR_ARG", -2: "DMALA_ERR_UNSUPPORTED", -3: "DMALA_ERR_NONFINITE",
          -4: "DMALA_ERR_WORKSPACE", -5: "DMALA_ERR_HIP"}


class Params(ctypes.Structure):
    _fields_ = [("n_chains", ctypes.c_int32), ("n_iters", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("precision", ctypes.c_int), ("proposal", ctypes.c_int), ("tau", ctypes.c_double),
                ("alpha_mult", ctypes.c_double), ("beta_mult", ctypes.c_double), ("gamma_mult", ctypes.c_double),
                ("tile_config", ctypes.c_int32), ("wg_chain_blocks", ctypes.c_int32),
                ("mlp_weights", ctypes.c_void_p), ("mix_eps", ctypes.c_double), ("llr_mode", ctypes.c_int),
                ("counter_base", ctypes.c_uint32)]


class Shape(ctypes.Structure):
    _fields_ = [("nt", ctypes.c_int32), ("nr", ctypes.c_int32), ("qam_order", ctypes.c_int32)]


class Outputs(ctypes.Structure):
    _fields_ = [("symbols", ctypes.c_void_p), ("marginals", ctypes.c_void_p), ("llrs", ctypes.c_void_p),
                ("best_energy", ctypes.c_void_p), ("final_state", ctypes.c_void_p), ("accept_count", ctypes.c_void_p),
                ("marginals_mc", ctypes.c_void_p), ("trace_accept", ctypes.c_void_p), ("trace_hash", ctypes.c_void_p),
                ("train_rows", ctypes.c_void_p), ("status", ctypes.c_void_p), ("stage_events", ctypes.c_void_p * 4)]


class DmalaError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS.get(status, status), msg))
        self.status = status


_lib = None


def lib():
    """The loaded library (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libdmala.so is not built (run paper_2407_06042_amd.build.build())")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_size_t
        L.dmala_workspace_size.restype = sz
        L.dmala_workspace_size.argtypes = [i32, i32, i32, i32, ctypes.POINTER(Params)]
        L.dmala_detect.restype = ctypes.c_int
        L.dmala_detect.argtypes = [vp, vp, vp, i32, i32, i32, i32, vp, ctypes.POINTER(Params),
                                   ctypes.POINTER(Outputs), vp, sz, vp]
        L.dmala_detect_static.restype = ctypes.c_int
        L.dmala_detect_static.argtypes = [vp, vp, vp, i32, i32, i32, i32, vp, ctypes.POINTER(Params),
                                          ctypes.POINTER(Outputs), vp]
        L.dmala_debug_eval.restype = ctypes.c_int
        L.dmala_debug_eval.argtypes = [vp, vp, vp, i32, i32, i32, i32, ctypes.POINTER(Params), vp, vp, i32, vp, vp, vp, sz,
                                       vp]
        L.dmala_gx_loop_sink_size.restype = sz
        L.dmala_gx_loop_sink_size.argtypes = [i32, i32, i32]
        L.dmala_gx_loop.restype = ctypes.c_int
        L.dmala_gx_loop.argtypes = [vp, vp, vp, i32, i32, i32, i32, ctypes.POINTER(Params), i32, i32, vp, vp, sz, vp]
        L.dmala_sync_status.restype = ctypes.c_int
        L.dmala_sync_status.argtypes = [vp, i32, vp]
        L.dmala_detect_one_workspace_size.restype = sz
        L.dmala_detect_one_workspace_size.argtypes = [i32, i32, i32, i32]
        L.dmala_detect_one.restype = ctypes.c_int
        L.dmala_detect_one.argtypes = [vp, vp, ctypes.c_float, i32, i32, vp, i32, i32, i32, ctypes.c_uint64, vp, vp, vp,
                                       sz, vp]
        L.dmala_plan_create.restype = ctypes.c_int
        L.dmala_plan_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(Shape), i32, ctypes.POINTER(Params),
                                        ctypes.POINTER(sz)]
        L.dmala_plan_execute.restype = ctypes.c_int
        L.dmala_plan_execute.argtypes = [vp, vp, vp, vp, ctypes.POINTER(Outputs), vp, sz, vp]
        L.dmala_plan_autotune.restype = ctypes.c_int
        L.dmala_plan_autotune.argtypes = [vp, vp, vp, vp, vp, sz, ctypes.c_char_p, vp]
        L.dmala_plan_num_classes.restype = i32
        L.dmala_plan_num_classes.argtypes = [vp]
        L.dmala_plan_class_info.restype = ctypes.c_int
        L.dmala_plan_class_info.argtypes = [vp, i32, ctypes.POINTER(Shape), ctypes.POINTER(i32), ctypes.POINTER(i32),
                                            ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_double)]
        L.dmala_plan_graph_info.restype = ctypes.c_int
        L.dmala_plan_graph_info.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32)]
        L.dmala_plan_destroy.restype = None
        L.dmala_plan_destroy.argtypes = [vp]
        L.dmala_mlp_forward.restype = ctypes.c_int
        L.dmala_mlp_forward.argtypes = [vp, vp, i32, i32, vp, vp]
        L.dmala_mlp_train_workspace_size.restype = sz
        L.dmala_mlp_train_workspace_size.argtypes = [i32]
        L.dmala_mlp_train_step.restype = ctypes.c_int
        L.dmala_mlp_train_step.argtypes = [vp, vp, vp, i32, ctypes.c_float, vp, vp, i32, vp, vp, vp, sz, vp]
        L.dmala_last_error.restype = ctypes.c_char_p
        L.dmala_version.restype = ctypes.c_char_p
        _lib = L
    return _lib


EXPORTED = ["dmala_workspace_size", "dmala_detect", "dmala_detect_static", "dmala_debug_eval", "dmala_sync_status",
            "dmala_detect_one_workspace_size", "dmala_detect_one", "dmala_gx_loop_sink_size", "dmala_gx_loop", "dmala_plan_create", "dmala_plan_execute",
            "dmala_plan_autotune", "dmala_plan_num_classes", "dmala_plan_class_info", "dmala_plan_graph_info",
            "dmala_plan_destroy",
            "dmala_mlp_forward", "dmala_mlp_train_workspace_size", "dmala_mlp_train_step",
            "dmala_last_error", "dmala_version"]


def last_error():
    return lib().dmala_last_error().decode()


LLR_MODES = {"is": 0, "list": 1, "mc": 2}


def make_params(n_chains, n_iters, seed, precision="fp32", proposal="precond", tau=2.0,
                alpha_mult=1.0, beta_mult=1.0, gamma_mult=1.0, tile_config=0, mlp_weights=None, mix_eps=0.0,
                llr_mode="is", counter_base=0):
    """mlp_weights: device float32 tensor of MLP_PARAMS values (learned proposal only)."""
    w = None
    if mlp_weights is not None:
        _check_weights(mlp_weights)
        w = mlp_weights.data_ptr()
    return Params(int(n_chains), int(n_iters), int(seed) & ((1 << 64) - 1), PRECISIONS[precision],
                  PROPOSALS[proposal], float(tau), float(alpha_mult), float(beta_mult), float(gamma_mult),
                  int(tile_config), 0, w, float(mix_eps), LLR_MODES[llr_mode], int(counter_base))


def _check_weights(w):
    import torch
    if not (isinstance(w, torch.Tensor) and w.is_cuda and w.dtype == torch.float32 and w.is_contiguous()
            and w.numel() == MLP_PARAMS):
        raise ValueError("mlp weights must be a contiguous float32 device tensor of %d values" % MLP_PARAMS)


def workspace_size(n_inst, nt, nr, M, params):
    n = lib().dmala_workspace_size(n_inst, nt, nr, M, ctypes.byref(params))
    if n == 0:
        raise DmalaError(-1, last_error())
    return n


def device_inputs(H, y, sigma2, precision="fp32", device="cuda"):
    """Marshal host arrays into the library's device layout.

    H: (B, Nr, Nt) complex, y: (B, Nr) complex, sigma2: (B,).  Returns torch
    tensors (Hcm, y, sigma2): Hcm is (B, Nt, Nr), i.e. column-major per instance.
    """
    import torch
    ct, rt = (np.complex128, np.float64) if precision == "fp64" else (np.complex64, np.float32)
    Hcm = np.ascontiguousarray(np.transpose(np.asarray(H), (0, 2, 1))).astype(ct)
    return (torch.from_numpy(Hcm).to(device), torch.from_numpy(np.ascontiguousarray(y).astype(ct)).to(device),
            torch.from_numpy(np.ascontiguousarray(sigma2).astype(rt)).to(device))


class Detector:
    """Reusable detector for one problem shape: owns a workspace and output tensors."""

    def __init__(self, n_inst, nt, nr, M, n_chains, n_iters, seed=0, precision="fp32", proposal="precond",
                 tau=2.0, alpha_mult=1.0, beta_mult=1.0, gamma_mult=1.0, device="cuda",
                 outputs=("symbols", "marginals", "llrs", "best_energy"), trace=False, tile_config=0,
                 mlp_weights=None, mix_eps=0.0, llr_mode="is", counter_base=0):
        import torch
        self.torch = torch
        self.n_inst, self.nt, self.nr, self.M = n_inst, nt, nr, M
        self.precision = precision
        self.mlp_weights = mlp_weights  # keeps the tensor alive while the detector holds its pointer
        self.params = make_params(n_chains, n_iters, seed, precision, proposal, tau, alpha_mult, beta_mult,
                                  gamma_mult, tile_config, mlp_weights, mix_eps, llr_mode, counter_base)
        self.ws_bytes = workspace_size(n_inst, nt, nr, M, self.params)
        self.ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=device)
        nb = int(round(np.log2(M)))
        shapes = dict(symbols=((n_inst, nt), torch.int32), marginals=((n_inst, nt, M), torch.float32),
                      llrs=((n_inst, nt, nb), torch.float32), best_energy=((n_inst,), torch.float32),
                      final_state=((n_inst, n_chains, 2 * nt), torch.int8),
                      accept_count=((n_inst, n_chains), torch.int32),
                      marginals_mc=((n_inst, nt, M), torch.float32),
                      train_rows=((n_inst, n_chains, nt, TRAIN_ROW), torch.float32),
                      status=((n_inst,), torch.int32))
        want = set(outputs)
        if trace:
            want |= {"final_state", "accept_count"}
        self.out = {k: torch.empty(s, dtype=d, device=device) for k, (s, d) in shapes.items() if k in want}
        if trace:
            self.out["trace_accept"] = torch.zeros((n_inst, n_chains, (n_iters + 31) // 32), dtype=torch.int32, device=device)
            self.out["trace_hash"] = torch.zeros((n_inst, n_chains, n_iters), dtype=torch.int32, device=device)
        o = Outputs()
        for name, _ in Outputs._fields_[:-1]:
            setattr(o, name, self.out[name].data_ptr() if name in self.out else None)
        self._outs = o

    def _ws_ptr(self):
        p = self.ws.data_ptr()
        return (p + 255) // 256 * 256

    def __call__(self, Hcm, y, sigma2, stream=None, events=None, static_scratch=False):
        """Enqueue detection on the current (or given) stream; returns the output dict.

        events: optional 4 raw hipEvent_t handles recorded around the three kernels.
        static_scratch: run dmala_detect_static (the library's fixed device array as
        workspace) instead of dmala_detect with this detector's workspace.
        """
        torch = self.torch
        self._check_inputs(Hcm, y, sigma2)
        s = stream if stream is not None else torch.cuda.current_stream().cuda_stream
        for i in range(4):
            self._outs.stage_events[i] = events[i] if events is not None else None
        if static_scratch:
            st = lib().dmala_detect_static(Hcm.data_ptr(), y.data_ptr(), sigma2.data_ptr(), self.n_inst, self.nt,
                                           self.nr, self.M, None, ctypes.byref(self.params), ctypes.byref(self._outs), s)
        else:
            st = lib().dmala_detect(Hcm.data_ptr(), y.data_ptr(), sigma2.data_ptr(), self.n_inst, self.nt, self.nr,
                                    self.M, None, ctypes.byref(self.params), ctypes.byref(self._outs), self._ws_ptr(),
                                    self.ws_bytes, s)
        if st != 0:
            raise DmalaError(st, last_error())
        return self.out

    def _check_inputs(self, Hcm, y, sigma2):
        torch = self.torch
        ct, rt = (torch.complex128, torch.float64) if self.precision == "fp64" else (torch.complex64, torch.float32)
        if Hcm.dtype != ct or y.dtype != ct or sigma2.dtype != rt:
            raise TypeError("inputs must be %s/%s for precision %s" % (ct, rt, self.precision))
        if tuple(Hcm.shape) != (self.n_inst, self.nt, self.nr) or tuple(y.shape) != (self.n_inst, self.nr) \
                or tuple(sigma2.shape) != (self.n_inst,):
            raise ValueError("input shapes do not match the detector")
        if not (Hcm.is_contiguous() and y.is_contiguous() and sigma2.is_contiguous()):
            raise ValueError("inputs must be contiguous")
        if not Hcm.is_cuda:
            raise ValueError("inputs must be device tensors")


def detect(Hcm, y, sigma2, M, n_chains, n_iters, seed, **kw):
    """One-shot detection (allocates a workspace).  See Detector for keywords."""
    n_inst, nt, nr = Hcm.shape
    d = Detector(n_inst, nt, nr, M, n_chains, n_iters, seed, device=Hcm.device, **kw)
    return d(Hcm, y, sigma2)


def debug_eval(Hcm, y, sigma2, M, x_from, x_to, precision="fp32", proposal="precond", tau=2.0,
               alpha_mult=1.0, beta_mult=1.0, gamma_mult=1.0, tile_config=0, mlp_weights=None, per_dim=False):
    """Transition quantities of the device chain for state pairs (see dmala_debug_eval).

    With proposal="learned" the quantities are those of the learned kernel alone.  per_dim=True
    returns (out, out_dim) with the per-dimension forward log q terms (n_inst, n_pairs, 2 Nt)."""
    import torch
    n_inst, nt, nr = Hcm.shape
    n_pairs = x_from.shape[1]
    p = make_params(n_pairs, 0, 0, precision, proposal, tau, alpha_mult, beta_mult, gamma_mult, tile_config,
                    mlp_weights, 0.0)
    ws_bytes = workspace_size(n_inst, nt, nr, M, p)
    ws = torch.empty(ws_bytes + 256, dtype=torch.uint8, device=Hcm.device)
    wp = (ws.data_ptr() + 255) // 256 * 256
    out = torch.empty((n_inst, n_pairs, 4), dtype=torch.float64, device=Hcm.device)
    od = torch.empty((n_inst, n_pairs, 2 * nt), dtype=torch.float64, device=Hcm.device) if per_dim else None
    xf = x_from.to(torch.int8).contiguous()
    xt = x_to.to(torch.int8).contiguous()
    st = lib().dmala_debug_eval(Hcm.data_ptr(), y.data_ptr(), sigma2.data_ptr(), n_inst, nt, nr, M, ctypes.byref(p),
                                xf.data_ptr(), xt.data_ptr(), n_pairs, out.data_ptr(),
                                od.data_ptr() if per_dim else None, wp, ws_bytes,
                                torch.cuda.current_stream().cuda_stream)
    if st != 0:
        raise DmalaError(st, last_error())
    return (out, od) if per_dim else out


class GxLoop:
    """The gradient contraction alone, looped (dmala_gx_loop): bf16 or fp16, preconditioned matrices."""

    def __init__(self, n_inst, nt, nr, M, n_chains, precision="bf16", device="cuda"):
        import torch
        self.torch = torch
        self.n_inst, self.nt, self.nr, self.M, self.C = n_inst, nt, nr, M, n_chains
        npad = 32
        while npad < 2 * nt:
            npad *= 2
        # the loop reads real-equivalent fragments: the layout it pins (1 + layout 0, 1, 3 or 4)
        tc = {32: 1, 64: 2, 128: 4, 256: 5}[npad]
        self.params = make_params(n_chains, 1, 0, precision, "precond", tile_config=tc)
        self.ws_bytes = workspace_size(n_inst, nt, nr, M, self.params)
        self.ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=device)
        self.sink = torch.zeros(lib().dmala_gx_loop_sink_size(n_inst, nt, n_chains), dtype=torch.float32,
                                device=device)

    def __call__(self, Hcm, y, sigma2, n_loops, run_setup=False):
        wp = (self.ws.data_ptr() + 255) // 256 * 256
        st = lib().dmala_gx_loop(Hcm.data_ptr(), y.data_ptr(), sigma2.data_ptr(), self.n_inst, self.nt, self.nr, self.M,
                                 ctypes.byref(self.params), int(n_loops), 1 if run_setup else 0, self.sink.data_ptr(),
                                 wp, self.ws_bytes, self.torch.cuda.current_stream().cuda_stream)
        if st != 0:
            raise DmalaError(st, last_error())
        return self.sink


def sync_status(status, stream=None):
    """dmala_sync_status on a device int32 status tensor: raises DmalaError(DMALA_ERR_NONFINITE) if any
    instance is flagged."""
    import torch
    s = stream if stream is not None else torch.cuda.current_stream().cuda_stream
    st = lib().dmala_sync_status(status.data_ptr(), status.numel(), s)
    if st != 0:
        raise DmalaError(st, last_error())


def detect_one(H, y, sigma2, M, n_chains, n_iters, seed, constellation=None, marginals=True):
    """dmala_detect_one: one problem, H (Nt, Nr) complex64 device tensor (column-major), y (Nr,) complex64
    device tensor, sigma2 a host float.  Synchronous; returns (symbols, marginals or None)."""
    import torch
    nt, nr = H.shape
    need = lib().dmala_detect_one_workspace_size(nt, nr, M, n_chains)
    if need == 0:
        raise DmalaError(-1, last_error())
    ws = torch.empty(need + 256, dtype=torch.uint8, device=H.device)
    wp = (ws.data_ptr() + 255) // 256 * 256
    sym = torch.empty(nt, dtype=torch.int32, device=H.device)
    marg = torch.empty((nt, M), dtype=torch.float32, device=H.device) if marginals else None
    pts = None
    if constellation is not None:
        c = np.ascontiguousarray(np.asarray(constellation, dtype=np.complex64))
        pts = c.ctypes.data_as(ctypes.c_void_p)
    st = lib().dmala_detect_one(H.data_ptr(), y.data_ptr(), float(sigma2), nt, nr, pts, M, n_chains, n_iters,
                                int(seed) & ((1 << 64) - 1), sym.data_ptr(), marg.data_ptr() if marginals else None,
                                wp, need, torch.cuda.current_stream().cuda_stream)
    if st != 0:
        raise DmalaError(st, last_error())
    return sym, marg


def pack_uneven(H_list, y_list, sigma2, precision="fp32", device="cuda"):
    """Pack per-instance host arrays (H_b: (Nr_b, Nt_b), y_b: (Nr_b,)) into the plan layout."""
    import torch
    ct, rt = (np.complex128, np.float64) if precision == "fp64" else (np.complex64, np.float32)
    Hp = np.concatenate([np.asarray(H).T.reshape(-1) for H in H_list]).astype(ct)   # column-major per instance
    yp = np.concatenate([np.asarray(y).reshape(-1) for y in y_list]).astype(ct)
    return (torch.from_numpy(Hp).to(device), torch.from_numpy(yp).to(device),
            torch.from_numpy(np.asarray(sigma2).astype(rt)).to(device))


class Plan:
    """Uneven batch (instances of different Nt, Nr, M) run as one graph launch."""

    def __init__(self, shapes, n_chains, n_iters, seed=0, precision="fp32", proposal="precond", tau=2.0,
                 device="cuda", outputs=("symbols", "marginals", "llrs", "best_energy", "final_state", "accept_count"),
                 mlp_weights=None, mix_eps=0.0):
        import torch
        self.torch = torch
        self.shapes = [tuple(int(v) for v in s) for s in shapes]
        n = len(self.shapes)
        arr = (Shape * n)(*[Shape(*s) for s in self.shapes])
        self.mlp_weights = mlp_weights
        self.params = make_params(n_chains, n_iters, seed, precision, proposal, tau, mlp_weights=mlp_weights,
                                  mix_eps=mix_eps)
        self.precision = precision
        h = ctypes.c_void_p()
        ws = ctypes.c_size_t()
        st = lib().dmala_plan_create(ctypes.byref(h), arr, n, ctypes.byref(self.params), ctypes.byref(ws))
        if st != 0:
            raise DmalaError(st, last_error())
        self.handle = h
        self.ws_bytes = ws.value
        self.ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=device)
        nt_sum = sum(s[0] for s in self.shapes)
        marg = sum(s[0] * s[2] for s in self.shapes)
        llr = sum(s[0] * int(round(np.log2(s[2]))) for s in self.shapes)
        sizes = dict(symbols=(nt_sum, torch.int32), marginals=(marg, torch.float32), llrs=(llr, torch.float32),
                     best_energy=(n, torch.float32), final_state=(n_chains * 2 * nt_sum, torch.int8),
                     accept_count=(n * n_chains, torch.int32), marginals_mc=(marg, torch.float32),
                     train_rows=(n_chains * nt_sum * TRAIN_ROW, torch.float32), status=(n, torch.int32),
                     trace_hash=(n * n_chains * max(1, n_iters), torch.int32),
                     trace_accept=(n * n_chains * ((n_iters + 31) // 32), torch.int32))
        self.out = {k: torch.empty(sizes[k][0], dtype=sizes[k][1], device=device) for k in outputs}
        o = Outputs()
        for name, _ in Outputs._fields_[:-1]:
            setattr(o, name, self.out[name].data_ptr() if name in self.out else None)
        self._outs = o

    def _ws_ptr(self):
        return (self.ws.data_ptr() + 255) // 256 * 256

    def __call__(self, H, y, sigma2, events=None):
        s = self.torch.cuda.current_stream().cuda_stream
        for i in range(4):
            self._outs.stage_events[i] = events[i] if events is not None else None
        st = lib().dmala_plan_execute(self.handle, H.data_ptr(), y.data_ptr(), sigma2.data_ptr(), ctypes.byref(self._outs),
                                      self._ws_ptr(), self.ws_bytes, s)
        if st != 0:
            raise DmalaError(st, last_error())
        return self.out

    def autotune(self, H, y, sigma2, cache_path=None):
        s = self.torch.cuda.current_stream().cuda_stream
        st = lib().dmala_plan_autotune(self.handle, H.data_ptr(), y.data_ptr(), sigma2.data_ptr(), self._ws_ptr(),
                                       self.ws_bytes, cache_path.encode() if cache_path else None, s)
        if st != 0:
            raise DmalaError(st, last_error())

    def classes(self):
        out = []
        for k in range(lib().dmala_plan_num_classes(self.handle)):
            sh, n, tc, cb, ms = Shape(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
            st = lib().dmala_plan_class_info(self.handle, k, ctypes.byref(sh), ctypes.byref(n), ctypes.byref(tc),
                                             ctypes.byref(cb), ctypes.byref(ms))
            if st != 0:
                raise DmalaError(st, last_error())
            out.append(dict(nt=sh.nt, nr=sh.nr, M=sh.qam_order, count=n.value, tile_config=tc.value,
                            wg_chain_blocks=cb.value, tuned_ms=ms.value))
        return out

    def graph_info(self):
        """(kernel nodes, persistent) of the plan's current graph; (-1, -1) before the first call."""
        nk, pe = ctypes.c_int32(), ctypes.c_int32()
        st = lib().dmala_plan_graph_info(self.handle, ctypes.byref(nk), ctypes.byref(pe))
        if st != 0:
            raise DmalaError(st, last_error())
        return nk.value, pe.value

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and _lib is not None:
            _lib.dmala_plan_destroy(h)
            self.handle = None


# ---------------------------------------------------------------- the learned proposal's network

def mlp_forward(weights, rows, row_stride=None):
    """Network outputs (R, 4) in the sampler's bf16 precision; rows: (R, >= 7) float32 device tensor."""
    import torch
    _check_weights(weights)
    rows = rows.contiguous()
    if rows.dtype != torch.float32 or not rows.is_cuda or rows.dim() != 2:
        raise ValueError("rows must be a 2-D float32 device tensor")
    R = rows.shape[0]
    out = torch.empty((R, 4), dtype=torch.float32, device=rows.device)
    st = lib().dmala_mlp_forward(weights.data_ptr(), rows.data_ptr(), R, rows.shape[1] if row_stride is None else row_stride,
                                 out.data_ptr(), torch.cuda.current_stream().cuda_stream)
    if st != 0:
        raise DmalaError(st, last_error())
    return out


class MlpTrainer:
    """Adam on the learned proposal's network with the library's training kernels.

    weights: float32 device tensor (updated in place).  Each step takes training
    rows (R, TRAIN_ROW) as exported by the sampler and int32 targets (R, 2)."""

    def __init__(self, weights, lr=1e-3):
        import torch
        _check_weights(weights)
        self.torch = torch
        self.w = weights
        self.m = torch.zeros_like(weights)
        self.v = torch.zeros_like(weights)
        self.lr = float(lr)
        self.t = 0
        self.ws = None
        self.ws_rows = 0
        self.loss = torch.zeros(1, dtype=torch.float32, device=weights.device)
        self.grad = torch.zeros_like(weights)

    def step(self, rows, targets, lr=None):
        torch = self.torch
        R = rows.shape[0]
        if tuple(rows.shape) != (R, TRAIN_ROW) or rows.dtype != torch.float32 or not rows.is_contiguous():
            raise ValueError("rows must be contiguous float32 (R, %d)" % TRAIN_ROW)
        if tuple(targets.shape) != (R, 2) or targets.dtype != torch.int32 or not targets.is_contiguous():
            raise ValueError("targets must be contiguous int32 (R, 2)")
        need = lib().dmala_mlp_train_workspace_size(R)
        if self.ws is None or self.ws.numel() < need + 256:
            self.ws = torch.empty(need + 256, dtype=torch.uint8, device=self.w.device)
        wp = (self.ws.data_ptr() + 255) // 256 * 256
        self.t += 1
        st = lib().dmala_mlp_train_step(self.w.data_ptr(), self.m.data_ptr(), self.v.data_ptr(), self.t,
                                        float(self.lr if lr is None else lr), rows.data_ptr(), targets.data_ptr(), R,
                                        self.loss.data_ptr(), self.grad.data_ptr(), wp, need,
                                        torch.cuda.current_stream().cuda_stream)
        if st != 0:
            raise DmalaError(st, last_error())
        return self.loss
