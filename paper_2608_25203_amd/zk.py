"""Thin ctypes binding of libzk.so (argument marshalling only).

The functions below carry the C ABI's names (include/zk.h) and pass device
pointers and the current torch stream straight through; every step of the
computation runs in the HIP library.  PyTorch is used only to own device
memory (fields and the workspace) and to name the stream.  There is no
fallback: if libzk.so is missing or fails to load, `lib()` raises.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libzk.so")

ZK_OK, ZK_EINVAL, ZK_ENOWS, ZK_EDEVICE, ZK_EDIVERGED = 0, -1, -2, -3, -4
ZK_OPT_EPS, ZK_OPT_TAPER, ZK_OPT_FILTER, ZK_OPT_PRECISION, ZK_OPT_CHECK, ZK_OPT_PROFILE = 1, 2, 3, 4, 5, 6
ZK_OPT_INTEGRATOR = 7
ZK_INTEGRATOR_RK4, ZK_INTEGRATOR_IFAB2 = 0, 1
ZK_OPT_BOUNDARY = 8
ZK_BC_PERIODIC, ZK_BC_REFLECT = 0, 1
ZK_OPT_ROW_FFT = 9
ZK_OPT_ROW_PROGRAMS = 10
ZK_ROW_FFT_STOCKHAM, ZK_ROW_FFT_LANES = 0, 1
ZK_KERNEL_ROW_PAD, ZK_KERNEL_ROW_BASE, ZK_KERNEL_COL_PAD, ZK_KERNEL_COL_BASE, ZK_KERNEL_REDUCE = 0, 1, 2, 3, 4
KERNEL_NAMES = {0: "row_pad", 1: "row_base", 2: "col_pad", 3: "col_base", 4: "reduce"}

EXPORTS = ("zk_create", "zk_destroy", "zk_set_option", "zk_get_option", "zk_workspace_bytes", "zk_bind", "zk_dtn",
           "zk_rhs", "zk_step", "zk_step_static", "zk_hamiltonian", "zk_kernel_stats", "zk_autotune", "zk_team_shape", "zk_inverse_dtn",
           "zk_depth_velocity", "zk_set_team_shape", "zk_last_error",
           "zk_cnn_create", "zk_cnn_destroy", "zk_cnn_workspace_bytes", "zk_cnn_bind", "zk_cnn_set_params",
           "zk_cnn_get_params", "zk_cnn_forward", "zk_cnn_gradient", "zk_cnn_train_step", "zk_cnn_last_error",
           "zk_closure_create", "zk_closure_destroy", "zk_closure_workspace_bytes", "zk_closure_bind",
           "zk_closure_dtn", "zk_closure_features", "zk_closure_crops", "zk_closure_step", "zk_closure_stats",
           "zk_closure_last_error",
           "zk_batch_create", "zk_batch_destroy", "zk_batch_workspace_bytes", "zk_batch_bind", "zk_batch_set_fields",
           "zk_batch_set_option", "zk_batch_step", "zk_batch_autotune", "zk_batch_tuning", "zk_batch_stats",
           "zk_batch_last_error")
ZK_BATCH_OPT_GRAPH = 1
ZK_BATCH_OPT_PERSISTENT = 2
ZK_STATIC_WS_BYTES = 64 << 20  # size of the library's fixed device scratch (zk.h)


class ZkTile(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("Lx", ctypes.c_double), ("Ly", ctypes.c_double),
                ("depth", ctypes.c_double), ("M", ctypes.c_int)]
ZK_CNN_NPARAMS = 19681

_lib = None


class ZKError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"zk error {code}: {msg}")
        self.code = code


def lib():
    """Load libzk.so once and declare the signatures of include/zk.h."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    L = ctypes.CDLL(LIB_PATH)
    vp, i, d, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
    L.zk_create.argtypes = [i, i, d, d, d, d, i]
    L.zk_create.restype = vp
    L.zk_destroy.argtypes = [vp]
    L.zk_destroy.restype = None
    L.zk_set_option.argtypes = [vp, i, d]
    L.zk_set_option.restype = i
    L.zk_get_option.argtypes = [vp, i, ctypes.POINTER(d)]
    L.zk_get_option.restype = i
    L.zk_workspace_bytes.argtypes = [vp]
    L.zk_workspace_bytes.restype = sz
    L.zk_bind.argtypes = [vp, vp, sz, vp]
    L.zk_bind.restype = i
    L.zk_dtn.argtypes = [vp, vp, vp, vp]
    L.zk_dtn.restype = i
    L.zk_rhs.argtypes = [vp, vp, vp, vp, vp]
    L.zk_rhs.restype = i
    L.zk_step.argtypes = [vp, vp, vp, d, i]
    L.zk_step.restype = i
    L.zk_step_static.argtypes = [vp, vp, vp, d, i, vp]
    L.zk_step_static.restype = i
    L.zk_hamiltonian.argtypes = [vp, vp, vp, ctypes.POINTER(d)]
    L.zk_hamiltonian.restype = i
    L.zk_kernel_stats.argtypes = [vp, i, ctypes.POINTER(d), ctypes.POINTER(d), ctypes.POINTER(d),
                                  ctypes.POINTER(ctypes.c_longlong)]
    L.zk_kernel_stats.restype = i
    L.zk_inverse_dtn.argtypes = [vp, vp, vp, vp, i]
    L.zk_inverse_dtn.restype = i
    L.zk_depth_velocity.argtypes = [vp, vp, vp, i, ctypes.POINTER(d), vp]
    L.zk_depth_velocity.restype = i
    L.zk_autotune.argtypes = [vp, d, i]
    L.zk_autotune.restype = i
    L.zk_set_team_shape.argtypes = [vp, i, i, i]
    L.zk_set_team_shape.restype = i
    L.zk_team_shape.argtypes = [vp, i, i, ctypes.POINTER(i), ctypes.POINTER(i)]
    L.zk_team_shape.restype = i
    L.zk_last_error.argtypes = [vp]
    L.zk_last_error.restype = ctypes.c_char_p
    ll, pd, pf = ctypes.c_longlong, ctypes.POINTER(d), ctypes.POINTER(ctypes.c_float)
    L.zk_cnn_create.argtypes = [ll]
    L.zk_cnn_create.restype = vp
    L.zk_cnn_destroy.argtypes = [vp]
    L.zk_cnn_destroy.restype = None
    L.zk_cnn_workspace_bytes.argtypes = [vp]
    L.zk_cnn_workspace_bytes.restype = sz
    L.zk_cnn_bind.argtypes = [vp, vp, sz, vp]
    L.zk_cnn_set_params.argtypes = [vp, pf]
    L.zk_cnn_get_params.argtypes = [vp, pf]
    L.zk_cnn_forward.argtypes = [vp, vp, vp, i, i, i]
    L.zk_cnn_gradient.argtypes = [vp, vp, i, i, i, i, pd, pf]
    L.zk_cnn_train_step.argtypes = [vp, vp, i, i, i, i, d, pd]
    for f in ("zk_cnn_bind", "zk_cnn_set_params", "zk_cnn_get_params", "zk_cnn_forward", "zk_cnn_gradient",
              "zk_cnn_train_step"):
        getattr(L, f).restype = i
    L.zk_cnn_last_error.argtypes = [vp]
    L.zk_cnn_last_error.restype = ctypes.c_char_p
    pll, pi = ctypes.POINTER(ll), ctypes.POINTER(i)
    L.zk_closure_create.argtypes = [vp, vp, vp, d, d, d]
    L.zk_closure_create.restype = vp
    L.zk_closure_destroy.argtypes = [vp]
    L.zk_closure_destroy.restype = None
    L.zk_closure_workspace_bytes.argtypes = [vp]
    L.zk_closure_workspace_bytes.restype = sz
    L.zk_closure_bind.argtypes = [vp, vp, sz]
    L.zk_closure_dtn.argtypes = [vp, vp, vp, vp]
    L.zk_closure_features.argtypes = [vp, vp, vp, vp]
    L.zk_closure_crops.argtypes = [vp, vp, pi, i, i, i, vp]
    L.zk_closure_step.argtypes = [vp, vp, vp, d, i, i, d]
    L.zk_closure_stats.argtypes = [vp, pll, pll, pll, pd, pd]
    for f in ("zk_closure_bind", "zk_closure_dtn", "zk_closure_features", "zk_closure_crops", "zk_closure_step",
              "zk_closure_stats"):
        getattr(L, f).restype = i
    L.zk_closure_last_error.argtypes = [vp]
    L.zk_closure_last_error.restype = ctypes.c_char_p
    L.zk_batch_create.argtypes = [i, ctypes.POINTER(ZkTile), d, i]
    L.zk_batch_create.restype = vp
    L.zk_batch_destroy.argtypes = [vp]
    L.zk_batch_destroy.restype = None
    L.zk_batch_workspace_bytes.argtypes = [vp]
    L.zk_batch_workspace_bytes.restype = sz
    L.zk_batch_bind.argtypes = [vp, vp, sz, vp]
    L.zk_batch_set_fields.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp)]
    L.zk_batch_set_option.argtypes = [vp, i, d]
    L.zk_batch_step.argtypes = [vp, d, i]
    L.zk_batch_autotune.argtypes = [vp, d, i]
    L.zk_batch_tuning.argtypes = [vp, i, pi, pi, pi, pi, pi]
    L.zk_batch_stats.argtypes = [vp, pll, pll]
    for f in ("zk_batch_bind", "zk_batch_set_fields", "zk_batch_set_option", "zk_batch_step", "zk_batch_autotune",
              "zk_batch_tuning", "zk_batch_stats"):
        getattr(L, f).restype = i
    L.zk_batch_last_error.argtypes = [vp]
    L.zk_batch_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def _check(ctx, rc):
    if rc != ZK_OK:
        raise ZKError(rc, lib().zk_last_error(ctx).decode())
    return rc


# ---- C-ABI mirrors --------------------------------------------------------------
def zk_create(nx, ny, Lx, Ly, depth, g, M):
    ctx = lib().zk_create(int(nx), int(ny), float(Lx), float(Ly), float(depth), float(g), int(M))
    if not ctx:
        raise ZKError(ZK_EINVAL, "zk_create rejected the arguments")
    return ctx


def zk_destroy(ctx):
    lib().zk_destroy(ctx)


def zk_set_option(ctx, key, value):
    return _check(ctx, lib().zk_set_option(ctx, int(key), float(value)))


def zk_get_option(ctx, key):
    v = ctypes.c_double(0.0)
    _check(ctx, lib().zk_get_option(ctx, int(key), ctypes.byref(v)))
    return v.value


def zk_workspace_bytes(ctx):
    return int(lib().zk_workspace_bytes(ctx))


def zk_bind(ctx, ws_ptr, nbytes, stream_ptr):
    return _check(ctx, lib().zk_bind(ctx, ws_ptr, nbytes, stream_ptr))


def zk_dtn(ctx, eta_ptr, psi_ptr, g_ptr):
    return _check(ctx, lib().zk_dtn(ctx, eta_ptr, psi_ptr, g_ptr))


def zk_rhs(ctx, eta_ptr, psi_ptr, eta_t_ptr, psi_t_ptr):
    return _check(ctx, lib().zk_rhs(ctx, eta_ptr, psi_ptr, eta_t_ptr, psi_t_ptr))


def zk_step(ctx, eta_ptr, psi_ptr, dt, nsteps):
    return _check(ctx, lib().zk_step(ctx, eta_ptr, psi_ptr, float(dt), int(nsteps)))


def zk_step_static(ctx, eta_ptr, psi_ptr, dt, nsteps, stream_ptr):
    """zk_step with the library's fixed device scratch as workspace (no zk_bind, no allocation)."""
    return _check(ctx, lib().zk_step_static(ctx, eta_ptr, psi_ptr, float(dt), int(nsteps), stream_ptr))


def zk_hamiltonian(ctx, eta_ptr, psi_ptr):
    h = ctypes.c_double(0.0)
    _check(ctx, lib().zk_hamiltonian(ctx, eta_ptr, psi_ptr, ctypes.byref(h)))
    return h.value


def zk_kernel_stats(ctx, kind):
    """(ms, bytes, flops, launches) accumulated for one kernel kind; kind=-1 resets."""
    ms, by, fl, n = ctypes.c_double(0), ctypes.c_double(0), ctypes.c_double(0), ctypes.c_longlong(0)
    if kind == -1:
        _check(ctx, lib().zk_kernel_stats(ctx, -1, None, None, None, None))
        return None
    _check(ctx, lib().zk_kernel_stats(ctx, int(kind), ctypes.byref(ms), ctypes.byref(by), ctypes.byref(fl),
                                      ctypes.byref(n)))
    return ms.value, by.value, fl.value, n.value


# ---- torch convenience wrapper -------------------------------------------------------
class Solver:
    """One context bound to a torch-owned workspace on the current stream.

    Fields are float64 CUDA tensors of shape (ny, nx), contiguous."""

    def __init__(self, nx, ny, Lx, Ly, depth, g, M, eps=1.0, taper=True, filt=True, precision=64,
                 check=True, device="cuda", integrator="rk4", boundary="periodic"):
        import torch

        self.torch = torch
        self.nx, self.ny = int(nx), int(ny)
        self.device = torch.device(device)
        self.ctx = zk_create(nx, ny, Lx, Ly, depth, g, M)
        zk_set_option(self.ctx, ZK_OPT_BOUNDARY, {"periodic": ZK_BC_PERIODIC, "reflect": ZK_BC_REFLECT}[boundary])
        zk_set_option(self.ctx, ZK_OPT_PRECISION, precision)
        zk_set_option(self.ctx, ZK_OPT_INTEGRATOR, {"rk4": ZK_INTEGRATOR_RK4, "ifab2": ZK_INTEGRATOR_IFAB2}[integrator])
        zk_set_option(self.ctx, ZK_OPT_EPS, eps)
        zk_set_option(self.ctx, ZK_OPT_TAPER, 1.0 if taper else 0.0)
        zk_set_option(self.ctx, ZK_OPT_FILTER, 1.0 if filt else 0.0)
        zk_set_option(self.ctx, ZK_OPT_CHECK, 1.0 if check else 0.0)
        nbytes = zk_workspace_bytes(self.ctx)
        with torch.cuda.device(self.device):
            self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
            off = (-self.ws.data_ptr()) % 256
            self.stream = torch.cuda.current_stream(self.device)
            zk_bind(self.ctx, self.ws.data_ptr() + off, nbytes, self.stream.cuda_stream)

    def _field(self, x):
        t = self.torch
        x = t.as_tensor(x, dtype=t.float64, device=self.device)
        if x.shape != (self.ny, self.nx):
            raise ValueError(f"field shape {tuple(x.shape)} != {(self.ny, self.nx)}")
        return x.contiguous()

    def dtn(self, eta, psi):
        eta, psi = self._field(eta), self._field(psi)
        out = self.torch.empty_like(eta)
        zk_dtn(self.ctx, eta.data_ptr(), psi.data_ptr(), out.data_ptr())
        return out

    def inverse_dtn(self, eta, v, iters=8):
        """psi from (eta, v = G(eta) psi): eight fixed-point iterations by default."""
        eta, v = self._field(eta), self._field(v)
        out = self.torch.empty_like(eta)
        _check(self.ctx, lib().zk_inverse_dtn(self.ctx, eta.data_ptr(), v.data_ptr(), out.data_ptr(), int(iters)))
        return out

    def depth_velocity(self, eta, psi, ys):
        """(u, v, w) at the depths ys below the flat reference plane, a
        [len(ys)][3][ny][nx] device tensor (x, vertical and y velocity)."""
        eta, psi = self._field(eta), self._field(psi)
        ys = [float(y) for y in ys]
        out = self.torch.empty((len(ys), 3) + tuple(eta.shape), dtype=eta.dtype, device=eta.device)
        arr = (ctypes.c_double * max(len(ys), 1))(*ys)
        _check(self.ctx, lib().zk_depth_velocity(self.ctx, eta.data_ptr(), psi.data_ptr(), len(ys), arr,
                                                  out.data_ptr()))
        return out

    def rhs(self, eta, psi):
        eta, psi = self._field(eta), self._field(psi)
        a, b = self.torch.empty_like(eta), self.torch.empty_like(eta)
        zk_rhs(self.ctx, eta.data_ptr(), psi.data_ptr(), a.data_ptr(), b.data_ptr())
        return a, b

    def step(self, eta, psi, dt, nsteps):
        """In place on the given tensors (they must already be contiguous float64 on the device)."""
        if eta.dtype != self.torch.float64 or not eta.is_contiguous() or not psi.is_contiguous():
            raise ValueError("step works in place on contiguous float64 device tensors")
        zk_step(self.ctx, eta.data_ptr(), psi.data_ptr(), dt, nsteps)
        return eta, psi

    def hamiltonian(self, eta, psi):
        eta, psi = self._field(eta), self._field(psi)
        return zk_hamiltonian(self.ctx, eta.data_ptr(), psi.data_ptr())

    def autotune(self, dt, reps=3):
        """Time the compiled team shapes of every pass kind on one step and keep the fastest."""
        _check(self.ctx, lib().zk_autotune(self.ctx, float(dt), int(reps)))
        return self.team_shapes()

    def set_team_shape(self, row, pad, T):
        """Team size T of one pass kind (0 = default)."""
        _check(self.ctx, lib().zk_set_team_shape(self.ctx, int(bool(row)), int(bool(pad)), int(T)))

    def team_shapes(self):
        out = {}
        for row in (1, 0):
            for pad in (1, 0):
                T, E = ctypes.c_int(0), ctypes.c_int(0)
                _check(self.ctx, lib().zk_team_shape(self.ctx, row, pad, ctypes.byref(T), ctypes.byref(E)))
                out[("row" if row else "col") + ("_pad" if pad else "_base")] = (T.value, E.value)
        return out

    def kernel_stats(self):
        """{kind name: (ms, bytes, flops, launches)} for launches timed so far."""
        return {KERNEL_NAMES[k]: zk_kernel_stats(self.ctx, k) for k in KERNEL_NAMES}

    def reset_stats(self):
        zk_kernel_stats(self.ctx, -1)

    def set_option(self, key, value):
        zk_set_option(self.ctx, key, value)

    def get_option(self, key):
        return zk_get_option(self.ctx, key)

    def close(self):
        if getattr(self, "ctx", None):
            zk_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---- closure network ------------------------------------------------------------------
def _cnn_check(net, rc):
    if rc != ZK_OK:
        raise ZKError(rc, lib().zk_cnn_last_error(net).decode())
    return rc


class Net:
    """The closure network (zk_cnn_*) bound to a torch-owned workspace.

    Samples are float32 CUDA tensors [B, 4, H, W] (planes 0..2 input,
    plane 3 target); parameters are float32 numpy vectors of ZK_CNN_NPARAMS."""

    def __init__(self, max_pixels, device="cuda"):
        import torch

        self.torch = torch
        self.device = torch.device(device)
        self.net = lib().zk_cnn_create(int(max_pixels))
        if not self.net:
            raise ZKError(ZK_EINVAL, "zk_cnn_create rejected max_pixels")
        nbytes = int(lib().zk_cnn_workspace_bytes(self.net))
        with torch.cuda.device(self.device):
            self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
            off = (-self.ws.data_ptr()) % 256
            self.stream = torch.cuda.current_stream(self.device)
            _cnn_check(self.net, lib().zk_cnn_bind(self.net, self.ws.data_ptr() + off, nbytes,
                                                   self.stream.cuda_stream))

    @staticmethod
    def _fp(a):
        import numpy as np

        a = np.ascontiguousarray(a, dtype=np.float32)
        return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))

    def _samples(self, s):
        t = self.torch
        if s.dtype != t.float32 or s.dim() != 4 or s.shape[1] != 4 or not s.is_contiguous():
            raise ValueError("samples must be a contiguous float32 tensor [B, 4, H, W]")
        return s

    def set_params(self, params):
        a, p = self._fp(params)
        if a.size != ZK_CNN_NPARAMS:
            raise ValueError("parameter vector has the wrong length")
        _cnn_check(self.net, lib().zk_cnn_set_params(self.net, p))

    def get_params(self):
        import numpy as np

        out = np.empty(ZK_CNN_NPARAMS, dtype=np.float32)
        _cnn_check(self.net, lib().zk_cnn_get_params(self.net, out.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
        return out

    def forward(self, samples):
        s = self._samples(samples)
        B, _, H, W = s.shape
        y = self.torch.empty((B, H, W), dtype=self.torch.float32, device=self.device)
        _cnn_check(self.net, lib().zk_cnn_forward(self.net, s.data_ptr(), y.data_ptr(), B, H, W))
        return y

    def gradient(self, samples, halo):
        import numpy as np

        s = self._samples(samples)
        B, _, H, W = s.shape
        loss = ctypes.c_double(0.0)
        g = np.empty(ZK_CNN_NPARAMS, dtype=np.float32)
        _cnn_check(self.net, lib().zk_cnn_gradient(self.net, s.data_ptr(), B, H, W, int(halo), ctypes.byref(loss),
                                                   g.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
        return loss.value, g

    def train_step(self, samples, halo, lr, want_loss=False):
        s = self._samples(samples)
        B, _, H, W = s.shape
        loss = ctypes.c_double(0.0)
        _cnn_check(self.net, lib().zk_cnn_train_step(self.net, s.data_ptr(), B, H, W, int(halo), float(lr),
                                                     ctypes.byref(loss) if want_loss else None))
        return loss.value if want_loss else None

    def close(self):
        if getattr(self, "net", None):
            lib().zk_cnn_destroy(self.net)
            self.net = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---- learned-closure stepper ----------------------------------------------------------
class Closure:
    """zk_closure_* over a low-order Solver, an optional full-order Solver
    (fallback and error reference) and a Net, all on one device stream."""

    def __init__(self, low, full, net, k0, eta_scale, out_scale):
        import torch

        self.torch = torch
        self.low, self.full, self.net_obj = low, full, net
        self.c = lib().zk_closure_create(low.ctx, full.ctx if full is not None else None, net.net, float(k0),
                                         float(eta_scale), float(out_scale))
        if not self.c:
            raise ZKError(ZK_EINVAL, "zk_closure_create rejected the arguments")
        nbytes = int(lib().zk_closure_workspace_bytes(self.c))
        self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=low.device)
        off = (-self.ws.data_ptr()) % 256
        self._check(lib().zk_closure_bind(self.c, self.ws.data_ptr() + off, nbytes))

    def _check(self, rc):
        if rc != ZK_OK:
            raise ZKError(rc, lib().zk_closure_last_error(self.c).decode())

    def dtn(self, eta, psi):
        eta, psi = self.low._field(eta), self.low._field(psi)
        out = self.torch.empty_like(eta)
        self._check(lib().zk_closure_dtn(self.c, eta.data_ptr(), psi.data_ptr(), out.data_ptr()))
        return out

    def features(self, eta, psi):
        eta, psi = self.low._field(eta), self.low._field(psi)
        out = self.torch.empty((4, self.low.ny, self.low.nx), dtype=self.torch.float32, device=self.low.device)
        self._check(lib().zk_closure_features(self.c, eta.data_ptr(), psi.data_ptr(), out.data_ptr()))
        return out

    def crops(self, samples, offsets, h, w):
        """samples: float32 [4, ny, nx] device tensor; offsets: int array [n, 2] (row, col)."""
        import numpy as np

        offs = np.ascontiguousarray(offsets, dtype=np.int32).reshape(-1, 2)
        out = self.torch.empty((offs.shape[0], 4, h, w), dtype=self.torch.float32, device=self.low.device)
        self._check(lib().zk_closure_crops(self.c, samples.data_ptr(),
                                           offs.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), offs.shape[0],
                                           int(h), int(w), out.data_ptr()))
        return out

    def step(self, eta, psi, dt, nsteps, audit_every=0, tol=0.0):
        """In place on contiguous float64 device tensors."""
        if eta.dtype != self.torch.float64 or not eta.is_contiguous() or not psi.is_contiguous():
            raise ValueError("step works in place on contiguous float64 device tensors")
        self._check(lib().zk_closure_step(self.c, eta.data_ptr(), psi.data_ptr(), float(dt), int(nsteps),
                                          int(audit_every), float(tol)))
        return eta, psi

    def stats(self):
        a, b, n = ctypes.c_longlong(0), ctypes.c_longlong(0), ctypes.c_longlong(0)
        e1, e2 = ctypes.c_double(0), ctypes.c_double(0)
        self._check(lib().zk_closure_stats(self.c, ctypes.byref(a), ctypes.byref(b), ctypes.byref(n),
                                           ctypes.byref(e1), ctypes.byref(e2)))
        return {"closure_steps": a.value, "fallback_steps": b.value, "audits": n.value, "last_err": e1.value,
                "max_err": e2.value}

    def close(self):
        if getattr(self, "c", None):
            lib().zk_closure_destroy(self.c)
            self.c = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---- batches of tiles ------------------------------------------------------------------
class Batch:
    """zk_batch_*: tiles given as dicts with nx, ny, Lx, Ly, depth (inf or <= 0:
    deep) and M; fields are registered once (contiguous float64 device
    tensors [ny, nx]) and stepped in place."""

    def __init__(self, tiles, g=9.81, precision=32, device="cuda", graph=True, persistent=False):
        import math

        import torch

        self.torch = torch
        self.device = torch.device(device)
        arr = (ZkTile * len(tiles))()
        for k, t in enumerate(tiles):
            dep = t.get("depth", math.inf)
            arr[k] = ZkTile(int(t["nx"]), int(t["ny"]), float(t["Lx"]), float(t["Ly"]),
                            float(dep) if dep is not None else math.inf, int(t["M"]))
        self.tiles = [dict(t) for t in tiles]
        self.b = lib().zk_batch_create(len(tiles), arr, float(g), int(precision))
        if not self.b:
            raise ZKError(ZK_EINVAL, "zk_batch_create rejected the tiles")
        self._check(lib().zk_batch_set_option(self.b, ZK_BATCH_OPT_GRAPH, 1.0 if graph else 0.0))
        self._check(lib().zk_batch_set_option(self.b, ZK_BATCH_OPT_PERSISTENT, 1.0 if persistent else 0.0))
        nbytes = int(lib().zk_batch_workspace_bytes(self.b))
        with torch.cuda.device(self.device):
            self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
            off = (-self.ws.data_ptr()) % 256
            self.stream = torch.cuda.current_stream(self.device)
            self._check(lib().zk_batch_bind(self.b, self.ws.data_ptr() + off, nbytes, self.stream.cuda_stream))
        self.fields = None

    def _check(self, rc):
        if rc != ZK_OK:
            raise ZKError(rc, lib().zk_batch_last_error(self.b).decode())

    def set_fields(self, etas, psis):
        t = self.torch
        for k, (e, p) in enumerate(zip(etas, psis)):
            shp = (self.tiles[k]["ny"], self.tiles[k]["nx"])
            for x in (e, p):
                if x.dtype != t.float64 or not x.is_contiguous() or tuple(x.shape) != shp:
                    raise ValueError(f"tile {k}: fields must be contiguous float64 tensors of shape {shp}")
        self.fields = (list(etas), list(psis))  # keep them alive
        n = len(etas)
        pe = (ctypes.c_void_p * n)(*[e.data_ptr() for e in etas])
        pp = (ctypes.c_void_p * n)(*[p.data_ptr() for p in psis])
        self._check(lib().zk_batch_set_fields(self.b, pe, pp))

    def step(self, dt, nsteps):
        self._check(lib().zk_batch_step(self.b, float(dt), int(nsteps)))

    def autotune(self, dt, reps=3):
        self._check(lib().zk_batch_autotune(self.b, float(dt), int(reps)))
        return self.tuning()

    def tuning(self):
        out, k = [], 0
        while True:
            v = [ctypes.c_int(0) for _ in range(5)]
            if lib().zk_batch_tuning(self.b, k, *[ctypes.byref(x) for x in v]) != ZK_OK:
                return out
            out.append({"row": bool(v[0].value), "pad": bool(v[1].value), "n": v[2].value, "T": v[3].value,
                        "E": v[4].value})
            k += 1

    def stats(self):
        a, b = ctypes.c_longlong(0), ctypes.c_longlong(0)
        self._check(lib().zk_batch_stats(self.b, ctypes.byref(a), ctypes.byref(b)))
        return {"phases_per_step": a.value, "launches_per_step": b.value}

    def close(self):
        if getattr(self, "b", None):
            lib().zk_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
