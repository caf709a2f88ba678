"""Python binding of libfraclap (MI355X / gfx950 fractional Laplacian solver).

Argument marshalling only: every step of the method runs in the HIP library
behind the C ABI declared in include/fraclap.h.  Device memory and streams
come from PyTorch (ROCm).  There is no CPU fallback: if the library is not
built or no GPU is present, every call raises.
"""
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfraclap.so")

FL_OK, FL_E_INVALID, FL_E_NOMEM, FL_E_HIP, FL_E_NOCONV, FL_E_BREAKDOWN, FL_E_UNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
FL_F64, FL_F32 = 0, 1
FL_PC_NONE, FL_PC_FD, FL_PC_LEARNED, FL_PC_SPECTRAL, FL_PC_MTILDE, FL_PC_FD_BOX, FL_PC_AUTO = 0, 1, 2, 3, 4, 5, 6
STATUS_NAMES = {0: "ok", -1: "invalid", -2: "nomem", -3: "hip", -4: "noconv", -5: "breakdown", -6: "unsupported"}

EXPORTED = ["fl_make_weights", "fl_op_constants", "fl_op_padded", "fl_op_plan", "fl_op_export", "fl_apply", "fl_precond",
            "fl_precond_spectral", "fl_precond_any", "fl_apply_noalloc", "fl_solve", "fl_step", "fl_solve_batched", "fl_step_batched", "fl_profile_pass", "fl_op_destroy",
            "fl_last_error", "fl_device_allocations", "fl_net_create", "fl_net_nparams", "fl_net_set_params", "fl_net_get_params",
            "fl_net_forward", "fl_net_grad", "fl_net_train", "fl_learned_pairs", "fl_net_profile", "fl_net_destroy"]


class FlError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"fraclap status {status} ({STATUS_NAMES.get(status, '?')}): {msg}")
        self.status = status


class WeightsOpts(ctypes.Structure):
    _fields_ = [("delta_over_h", ctypes.c_double), ("dst_mode", ctypes.c_int), ("col_lanes", ctypes.c_int),
                ("sine_col_lanes", ctypes.c_int), ("reserved", ctypes.c_int * 3)]


class SolveOpts(ctypes.Structure):
    _fields_ = [("pc", ctypes.c_int), ("mixed", ctypes.c_int), ("maxit", ctypes.c_int),
                ("inner_tol", ctypes.c_double), ("use_x0", ctypes.c_int), ("graph", ctypes.c_int),
                ("poll_every", ctypes.c_int), ("max_outer", ctypes.c_int), ("net", ctypes.c_void_p)]


class Info(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("outer_iters", ctypes.c_int), ("status", ctypes.c_int),
                ("fell_back", ctypes.c_int), ("rel_res_true", ctypes.c_double),
                ("rel_res_recur", ctypes.c_double), ("ms", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def load(path=LIB_PATH):
    """Load the built library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise FileNotFoundError(f"{path} is missing: run __graft_entry__.build() (hipcc, gfx950) first")
    lib = ctypes.CDLL(path)
    P, I, D, I64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_int64
    sig = {
        "fl_make_weights": [I, D, D, ctypes.POINTER(I64), ctypes.POINTER(WeightsOpts), P, ctypes.POINTER(P)],
        "fl_op_constants": [P, ctypes.POINTER(D)],
        "fl_op_padded": [P, ctypes.POINTER(I64)],
        "fl_op_plan": [P, ctypes.POINTER(I64)],
        "fl_op_export": [P, I, P],
        "fl_apply": [P, P, P, I, I64, P, D, D],
        "fl_precond": [P, P, P, I, I64, P, D, D],
        "fl_precond_spectral": [P, P, P, I, I64, P, D, D],
        "fl_precond_any": [P, I, P, P, I, I64, P, D, D],
        "fl_apply_noalloc": [P, P, P, I, I64, P, D, D],
        "fl_solve": [P, P, P, D, ctypes.POINTER(SolveOpts), P, ctypes.POINTER(Info)],
        "fl_step": [P, P, D, D, P, P, P, D, ctypes.POINTER(SolveOpts), ctypes.POINTER(Info)],
        "fl_solve_batched": [I, ctypes.POINTER(P), ctypes.POINTER(P), ctypes.POINTER(P), ctypes.POINTER(D),
                             ctypes.POINTER(SolveOpts), ctypes.POINTER(P), ctypes.POINTER(Info)],
        "fl_step_batched": [I, ctypes.POINTER(P), ctypes.POINTER(P), ctypes.POINTER(D), D, I, D,
                            ctypes.POINTER(SolveOpts), ctypes.POINTER(Info)],
        "fl_profile_pass": [P, I, I, I, ctypes.POINTER(D)],
        "fl_op_destroy": [P],
        "fl_last_error": [],
        "fl_device_allocations": [],
        "fl_net_create": [I, P, ctypes.POINTER(P)],
        "fl_net_nparams": [I],
        "fl_net_set_params": [P, P],
        "fl_net_get_params": [P, P],
        "fl_net_forward": [P, P, ctypes.POINTER(D), P, I, I, I, I],
        "fl_net_grad": [P, P, ctypes.POINTER(D), P, P, I, I, I, I],
        "fl_net_train": [P, P, P, P, I, I, I, I, ctypes.POINTER(I), I, I, D, ctypes.POINTER(ctypes.c_float)],
        "fl_learned_pairs": [P, P, I64, P, I, P, P, I, I, I],
        "fl_net_profile": [P, I, I, I, I, I, ctypes.POINTER(D)],
        "fl_net_destroy": [P],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = {"fl_last_error": ctypes.c_char_p, "fl_net_nparams": ctypes.c_int64,
                      "fl_device_allocations": ctypes.c_int64}.get(name, ctypes.c_int)
    _lib = lib
    return lib


def device_allocations():
    """Device allocations the library has made so far in this process."""
    return int(load().fl_device_allocations())


def _check(status):
    if status != FL_OK:
        raise FlError(status, load().fl_last_error().decode())


def _ptr(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _need(t, dtype, numel=None, name="tensor"):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} has {t.numel()} elements, expected {numel}")
    return t


def solve_opts(pc=FL_PC_FD, mixed=0, maxit=0, inner_tol=0.0, use_x0=0, graph=1, poll_every=8, max_outer=0,
               net=None):
    """Solver options; net is a Net (needed for pc=FL_PC_LEARNED)."""
    o = SolveOpts(pc, mixed, maxit, inner_tol, use_x0, graph, poll_every, max_outer, None)
    if net is not None:
        o.net = net._h.value
        o._keep = net  # keep the network alive as long as the options
    return o


class Op:
    """fl_op handle: the discrete fractional Laplacian M on an n_1 x ... x n_d grid."""

    def __init__(self, d, alpha, h, n, delta_over_h=20.0, stream=None, dst_mode=0, col_lanes=0, sine_col_lanes=0):
        lib = load()
        self.d, self.alpha, self.h = int(d), float(alpha), float(h)
        self.n = tuple(int(v) for v in (n if hasattr(n, "__len__") else [n] * d))
        if len(self.n) != self.d:
            raise ValueError("len(n) must equal d")
        if stream is None:
            # a private stream of default priority: hipGraph capture needs a non-null stream
            stream = torch.cuda.Stream()
        self.stream = stream
        arr = (ctypes.c_int64 * 3)(*(list(self.n) + [1] * (3 - self.d)))
        opts = WeightsOpts(delta_over_h, dst_mode, col_lanes, sine_col_lanes, (ctypes.c_int * 3)())
        h_ = ctypes.c_void_p()
        _check(lib.fl_make_weights(self.d, self.alpha, self.h, arr, ctypes.byref(opts),
                                   ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h_)))
        self._h = h_
        self.N = 1
        for v in self.n:
            self.N *= v

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            load().fl_op_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def constants(self):
        out = (ctypes.c_double * 8)()
        _check(load().fl_op_constants(self._h, out))
        return dict(zip(["C", "Z", "B", "a2", "a3s", "omega0", "omega_e", "Chma"], list(out)))

    def padded(self):
        out = (ctypes.c_int64 * 3)()
        _check(load().fl_op_padded(self._h, out))
        return tuple(out[i] for i in range(self.d))

    def plan(self):
        """Plans: {"f64"/"f32": [(sine form, length) per axis], "col_lanes": lanes per column of the symbol pass};
        sine form 1 direct, 2 chirp-z, 3 prime form (n + 1 = 257); col lanes 0 = run-time plan."""
        out = (ctypes.c_int64 * 16)()
        _check(load().fl_op_plan(self._h, out))
        plan = {p: [(int(out[3 * i + a]), int(out[6 + 3 * i + a])) for a in range(self.d)]
                for i, p in enumerate(("f64", "f32"))}
        plan["col_lanes"] = {"f64": int(out[12]), "f32": int(out[13])}
        plan["sine_col_lanes"] = {"f64": int(out[14]), "f32": int(out[15])}
        return plan

    def export(self, which):
        shape = tuple(p // 2 + 1 for p in self.padded())
        t = torch.empty(shape, dtype=torch.float32 if which == 2 else torch.float64, device="cuda")
        _check(load().fl_op_export(self._h, which, _ptr(t)))
        self.stream.synchronize()
        return t

    def profile_pass(self, dtype, which, reps=50):
        """Average ms per launch of one pass (HIP events on the op stream)."""
        ms = ctypes.c_double()
        _check(load().fl_profile_pass(self._h, FL_F64 if dtype == torch.float64 else FL_F32, which, reps,
                                      ctypes.byref(ms)))
        return ms.value

    def _enter(self):
        self.stream.wait_stream(torch.cuda.current_stream())

    def _leave(self):
        torch.cuda.current_stream().wait_stream(self.stream)

    def _batch(self, u):
        if u.numel() % self.N:
            raise ValueError("input size is not a multiple of the grid size")
        return u.numel() // self.N

    def apply(self, u, mask=None, shift0=0.0, shift1=1.0, out=None):
        dt = FL_F64 if u.dtype == torch.float64 else FL_F32
        _need(u, u.dtype, name="u")
        if u.dtype not in (torch.float64, torch.float32):
            raise ValueError("u must be float64 or float32")
        _need(mask, torch.uint8, self.N, "mask")
        out = torch.empty_like(u) if out is None else _need(out, u.dtype, u.numel(), "out")
        self._enter()
        _check(load().fl_apply(self._h, _ptr(u), _ptr(out), dt, self._batch(u), _ptr(mask), shift0, shift1))
        self._leave()
        return out

    def apply_noalloc(self, u, out, mask=None, shift0=0.0, shift1=1.0):
        """As apply, through fl_apply_noalloc (no device allocation; `out` must be given)."""
        dt = FL_F64 if u.dtype == torch.float64 else FL_F32
        _need(u, u.dtype, name="u")
        _need(out, u.dtype, u.numel(), "out")
        _need(mask, torch.uint8, self.N, "mask")
        self._enter()
        _check(load().fl_apply_noalloc(self._h, _ptr(u), _ptr(out), dt, self._batch(u), _ptr(mask), shift0, shift1))
        self._leave()
        return out

    def precond(self, r, mask=None, p0=0.0, p1=1.0, out=None, kind=FL_PC_FD):
        """z = (p0 I + p1 P)^{-1} r; P the FD Laplacian preconditioner (kind =
        FL_PC_FD, exact on a mask), the sine-basis diagonal of M (FL_PC_SPECTRAL),
        M~ (FL_PC_MTILDE, exact on a mask) or the box FD inverse restricted to a
        mask (FL_PC_FD_BOX)."""
        dt = FL_F64 if r.dtype == torch.float64 else FL_F32
        _need(r, r.dtype, name="r")
        _need(mask, torch.uint8, self.N, "mask")
        out = torch.empty_like(r) if out is None else _need(out, r.dtype, r.numel(), "out")
        if kind not in (FL_PC_FD, FL_PC_SPECTRAL, FL_PC_MTILDE, FL_PC_FD_BOX):
            raise ValueError("kind must be FL_PC_FD, FL_PC_SPECTRAL, FL_PC_MTILDE or FL_PC_FD_BOX")
        self._enter()
        if kind == FL_PC_FD:
            st = load().fl_precond(self._h, _ptr(r), _ptr(out), dt, self._batch(r), _ptr(mask), p0, p1)
        elif kind == FL_PC_SPECTRAL:
            st = load().fl_precond_spectral(self._h, _ptr(r), _ptr(out), dt, self._batch(r), _ptr(mask), p0, p1)
        else:
            st = load().fl_precond_any(self._h, kind, _ptr(r), _ptr(out), dt, self._batch(r), _ptr(mask), p0, p1)
        _check(st)
        self._leave()
        return out

    def tau(self, dtype=torch.float64):
        """Sine-basis diagonal of M, shape n (index k - 1)."""
        t = torch.empty(self.n, dtype=dtype, device="cuda")
        _check(load().fl_op_export(self._h, 3 if dtype == torch.float64 else 4, _ptr(t)))
        self.stream.synchronize()
        return t

    def solve(self, f, mask=None, tol=1e-10, opts=None, u=None, check=True):
        _need(f, torch.float64, self.N, "f")
        _need(mask, torch.uint8, self.N, "mask")
        u = torch.zeros_like(f) if u is None else _need(u, torch.float64, self.N, "u")
        info = Info()
        self._enter()
        st = load().fl_solve(self._h, _ptr(f), _ptr(mask), tol, ctypes.byref(opts or solve_opts()), _ptr(u),
                             ctypes.byref(info))
        if check:
            _check(st)
        return u, info.as_dict()

    def step(self, u, dt, theta=1.0, f_k=None, f_k1=None, mask=None, tol=1e-10, opts=None, check=True):
        _need(u, torch.float64, self.N, "u")
        _need(f_k, torch.float64, self.N, "f_k")
        _need(f_k1, torch.float64, self.N, "f_k1")
        _need(mask, torch.uint8, self.N, "mask")
        info = Info()
        self._enter()
        st = load().fl_step(self._h, _ptr(u), dt, theta, _ptr(f_k), _ptr(f_k1), _ptr(mask), tol,
                            ctypes.byref(opts or solve_opts()), ctypes.byref(info))
        if check:
            _check(st)
        return u, info.as_dict()


def _batch_common(ops):
    if not ops:
        raise ValueError("a batch needs at least one problem")
    st = ops[0].stream
    if any(o.stream.cuda_stream != st.cuda_stream for o in ops):
        raise ValueError("batched problems must share one stream: create their ops with the same stream=")
    if any(o.d != ops[0].d for o in ops):
        raise ValueError("batched problems must share the dimension d")
    ops[0]._enter()
    P = ctypes.c_void_p
    return P, (P * len(ops))(*[o._h for o in ops])


def solve_batched(ops, fs, tol=1e-10, opts=None, masks=None, us=None, check=True):
    """Solve ops[i] u_i = fs[i] for every i, all problems per launch (FP64 in/out);
    tol is one tolerance for all or a sequence of one per problem."""
    lib = load()
    k = len(ops)
    if len(fs) != k:
        raise ValueError("one right-hand side per op")
    for i, (o, f) in enumerate(zip(ops, fs)):
        _need(f, torch.float64, o.N, f"f[{i}]")
        if masks is not None:
            _need(masks[i], torch.uint8, o.N, f"mask[{i}]")
    us = us if us is not None else [torch.zeros_like(f) for f in fs]
    for i, (o, u) in enumerate(zip(ops, us)):
        _need(u, torch.float64, o.N, f"u[{i}]")
    P, hops = _batch_common(ops)
    hf = (P * k)(*[f.data_ptr() for f in fs])
    hm = (P * k)(*[0 if (masks is None or masks[i] is None) else masks[i].data_ptr() for i in range(k)])
    hu = (P * k)(*[u.data_ptr() for u in us])
    infos = (Info * k)()
    tols = [float(t) for t in tol] if hasattr(tol, "__len__") else [float(tol)] * k
    if len(tols) != k:
        raise ValueError("one tolerance per problem")
    htol = (ctypes.c_double * k)(*tols)
    st = lib.fl_solve_batched(k, hops, hf, hm, htol, ctypes.byref(opts or solve_opts()), hu, infos)
    if check:
        _check(st)
    return us, [i.as_dict() for i in infos]


def step_batched(ops, us, dts, theta=1.0, nsteps=1, tol=1e-10, opts=None, check=True):
    """Advance every problem by nsteps implicit theta steps (zero forcing), in place."""
    lib = load()
    k = len(ops)
    if len(us) != k or len(dts) != k:
        raise ValueError("one state and one dt per op")
    for i, (o, u) in enumerate(zip(ops, us)):
        _need(u, torch.float64, o.N, f"u[{i}]")
    P, hops = _batch_common(ops)
    hu = (P * k)(*[u.data_ptr() for u in us])
    hdt = (ctypes.c_double * k)(*[float(v) for v in dts])
    infos = (Info * k)()
    st = lib.fl_step_batched(k, hops, hu, hdt, theta, nsteps, tol, ctypes.byref(opts or solve_opts()), infos)
    if check:
        _check(st)
    return us, [i.as_dict() for i in infos]


class Net:
    """fl_net handle: the learned preconditioner's network for d = 2 (3 x 3
    kernels) or d = 3 (3 x 3 x 3), parameters on the device."""

    def __init__(self, stream=None, params=None, d=2):
        lib = load()
        if stream is None:
            stream = torch.cuda.Stream()
        self.stream = stream
        self.d = int(d)
        h_ = ctypes.c_void_p()
        _check(lib.fl_net_create(self.d, ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h_)))
        self._h = h_
        self.nparams = int(lib.fl_net_nparams(self.d))
        if params is not None:
            self.set_params(params)

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            load().fl_net_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _enter(self):
        self.stream.wait_stream(torch.cuda.current_stream())

    def _leave(self):
        torch.cuda.current_stream().wait_stream(self.stream)

    def _grid(self, x):
        """(batch, D, H, W) of x [B, H, W] (2D) or [B, D, H, W] (3D); an unbatched grid gains B = 1."""
        if x.dim() == self.d:
            x = x[None]
        if x.dim() != self.d + 1:
            raise ValueError(f"a {self.d}D network takes [B, {'D, ' if self.d == 3 else ''}H, W] grids")
        dims = tuple(x.shape)
        return x, (dims if self.d == 3 else (dims[0], 1) + dims[1:])

    def set_params(self, params):
        p = torch.as_tensor(params, dtype=torch.float32).to("cuda").contiguous()
        _need(p, torch.float32, self.nparams, "params")
        self._enter()
        _check(load().fl_net_set_params(self._h, _ptr(p)))

    def get_params(self):
        p = torch.empty(self.nparams, dtype=torch.float32, device="cuda")
        self._enter()
        _check(load().fl_net_get_params(self._h, _ptr(p)))
        return p

    def forward(self, x, alpha):
        """y = N(x, alpha) for x FP32 [B, (D,) H, W] (device); alpha: float or list of B floats."""
        _need(x, torch.float32, name="x")
        x, (B, D, H, W) = self._grid(x)
        al = [float(alpha)] * B if not hasattr(alpha, "__len__") else [float(a) for a in alpha]
        y = torch.empty_like(x)
        self._enter()
        _check(load().fl_net_forward(self._h, _ptr(x), (ctypes.c_double * B)(*al), _ptr(y), B, D, H, W))
        self._leave()
        return y

    def grad(self, x, alpha, gy):
        """d/dtheta sum(gy * N(x, alpha)) as an FP32 device vector."""
        _need(x, torch.float32, name="x")
        _need(gy, torch.float32, x.numel(), "gy")
        x, (B, D, H, W) = self._grid(x)
        al = [float(alpha)] * B if not hasattr(alpha, "__len__") else [float(a) for a in alpha]
        g = torch.empty(self.nparams, dtype=torch.float32, device="cuda")
        self._enter()
        _check(load().fl_net_grad(self._h, _ptr(x), (ctypes.c_double * B)(*al), _ptr(gy), _ptr(g), B, D, H, W))
        self._leave()
        return g

    def profile(self, which, H, W, reps=20, D=1):
        """Average ms per launch (HIP events on the net stream): 0 forward, 1 level-0 conv, 2 input, 3 output layer."""
        ms = ctypes.c_double()
        _check(load().fl_net_profile(self._h, which, D, H, W, reps, ctypes.byref(ms)))
        return ms.value

    def train(self, R, T, A, idx, batch, lr=1e-3):
        """Adam steps over minibatches idx (int array [steps, batch]); returns the loss per step."""
        _need(R, torch.float32, name="R")
        _need(T, torch.float32, R.numel(), "T")
        _need(A, torch.float32, R.shape[0], "A")
        import numpy as np
        idx = np.ascontiguousarray(np.asarray(idx, dtype=np.int32).reshape(-1, batch))
        steps = idx.shape[0]
        losses = (ctypes.c_float * max(steps, 1))()
        _, (npairs, D, H, W) = self._grid(R)
        self._enter()
        _check(load().fl_net_train(self._h, _ptr(R), _ptr(T), _ptr(A), npairs, D, H, W,
                                   idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), steps, batch, lr, losses))
        return [losses[i] for i in range(steps)]


def padded_grid(op):
    """The op's grid rounded up to multiples of 8 per side (the network grid)."""
    return tuple((v + 7) // 8 * 8 for v in op.n)


def learned_pairs(op, e, e_sub=None, padded=None):
    """Training pairs (R, T) of the learned preconditioner from FP64 errors
    e - e_sub: e is one grid (repeated) or [count, *n]; e_sub None or [count, *n].
    R, T: FP32 [count, *padded] (default: padded_grid(op))."""
    _need(e, torch.float64, name="e")
    if e.numel() == op.N and e_sub is not None:
        stride, count = 0, e_sub.numel() // op.N
    else:
        stride, count = op.N, e.numel() // op.N
    if count < 1 or e.numel() % op.N:
        raise ValueError("e must hold grids of the op")
    if e_sub is not None:
        _need(e_sub, torch.float64, count * op.N, "e_sub")
    pad = tuple(padded) if padded is not None else padded_grid(op)
    if len(pad) != op.d:
        raise ValueError("padded grid must have one side per axis")
    R = torch.empty((count,) + pad, dtype=torch.float32, device="cuda")
    T = torch.empty_like(R)
    Dp, Hp, Wp = pad if op.d == 3 else (1,) + pad
    op._enter()
    _check(load().fl_learned_pairs(op._h, _ptr(e), stride, _ptr(e_sub), count, _ptr(R), _ptr(T), Dp, Hp, Wp))
    op._leave()
    return R, T
