"""Python binding of the MI355X pressure-Poisson library (libcfdmi.so).

Argument marshalling only: every step of the solver, the time step and the
warm-start network runs in the library's HIP kernels.  torch tensors supply
device memory and the current stream.  If the library has not been built,
every call raises ImportError -- there is no fallback implementation.

Main entry points (names follow include/cfdmi.h):
    assemble(n_or_dims, pin=0) -> Csr
    rhs_prepare(A, b)
    solve(A, b, x0=None, tol=1e-10, precision="fp64", net=None, ...) -> (x, info)
    spmv(A, x) -> y
    State / step(state, dt, ...)
    Net (create, forward, train_step, gradient, params)
"""
from __future__ import annotations

import ctypes

from . import _lib
from ._lib import CfdError, CfdGrid, CfdSolveInfo, CfdSolveOpts, CfdState, check, load

PREC = {"fp64": 0, "mixed": 1}
FORM = {"pinned": 0, "projected": 1}
PRECOND = {"none": 0, "dic": 1}


def _torch():
    import torch
    return torch


def _stream():
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t, dtype, numel, name):
    torch = _torch()
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements, got {t.numel()}")
    return ctypes.c_void_p(t.data_ptr())


def make_grid(dims, h=None) -> CfdGrid:
    if isinstance(dims, int):
        dims = (dims, dims, dims)
    nx, ny, nz = (int(d) for d in dims)
    if h is None:
        h = 1.0 / max(nx, ny, nz)
    return CfdGrid(nx, ny, nz, float(h))


class Csr:
    """Device CSR matrix owned by the library (cfd_assemble / cfd_csr_destroy)."""

    def __init__(self, dims, pin=0, h=None):
        lib = load()
        self.grid = make_grid(dims, h)
        self.dims = (self.grid.nx, self.grid.ny, self.grid.nz)
        self.pin = int(pin)
        self._h = ctypes.c_void_p()
        check(lib.cfd_assemble(ctypes.byref(self.grid), self.pin, _stream(), ctypes.byref(self._h)))
        n, nnz = ctypes.c_int64(), ctypes.c_int64()
        check(lib.cfd_csr_info(self._h, ctypes.byref(n), ctypes.byref(nnz)))
        self.n, self.nnz = n.value, nnz.value

    @property
    def handle(self):
        return self._h

    def export(self):
        torch = _torch()
        rp = torch.empty(self.n + 1, dtype=torch.int32, device="cuda")
        col = torch.empty(self.nnz, dtype=torch.int32, device="cuda")
        val = torch.empty(self.nnz, dtype=torch.float64, device="cuda")
        check(load().cfd_csr_export(self._h, _ptr(rp, torch.int32, None, "row_ptr"),
                                    _ptr(col, torch.int32, None, "col"), _ptr(val, torch.float64, None, "val"),
                                    _stream()))
        return rp, col, val

    def close(self):
        if self._h:
            load().cfd_csr_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def assemble(dims, pin=0, h=None) -> Csr:
    return Csr(dims, pin, h)


def spmv(A: Csr, x, y=None, precision=None):
    torch = _torch()
    prec = precision if precision is not None else (1 if x.dtype == torch.float32 else 0)
    dt = torch.float32 if prec == 1 else torch.float64
    if y is None:
        y = torch.empty(A.n, dtype=dt, device=x.device)
    check(load().cfd_spmv(A.handle, prec, _ptr(x, dt, A.n, "x"), _ptr(y, dt, A.n, "y"), _stream()))
    return y


def spmv_sym(A: Csr, x, y=None, precision=None):
    """y = A x from the symmetric (diagonal + upper triangle) storage
    (cfd_spmv_sym); same arguments and result bits as spmv()."""
    torch = _torch()
    prec = precision if precision is not None else (1 if x.dtype == torch.float32 else 0)
    dt = torch.float32 if prec == 1 else torch.float64
    if y is None:
        y = torch.empty(A.n, dtype=dt, device=x.device)
    check(load().cfd_spmv_sym(A.handle, prec, _ptr(x, dt, A.n, "x"), _ptr(y, dt, A.n, "y"), _stream()))
    return y


def rhs_prepare(A: Csr, b):
    torch = _torch()
    check(load().cfd_rhs_prepare(A.handle, _ptr(b, torch.float64, A.n, "b"), _stream()))
    return b


def rhs_prepare_noalloc(A: Csr, b):
    """cfd_rhs_prepare_noalloc: rhs_prepare with the library's fixed scratch
    array (no device allocation)."""
    torch = _torch()
    check(load().cfd_rhs_prepare_noalloc(A.handle, _ptr(b, torch.float64, A.n, "b"), _stream()))
    return b


DRIVER = {"auto": 0, "steps": 1, "persistent": 2, "resident": 3}


def solve_opts(precision="fp64", max_iters=0, ru_delta=0.0, net=None, chunk=0, timing=False, formulation="pinned",
               precond="none", debug_breakdown_at=0, stop_margin=0.0, driver="auto", barrier_spins=0):
    """cfd_solve_opts; precond "dic" = the DIC preconditioner in red-black order;
    stop_margin <= 0: the library's default (0.05 mixed, 1 float64); driver
    "auto", "steps" (one launch per step) or "persistent" (one cooperative
    launch)."""
    return CfdSolveOpts(PREC[precision] if isinstance(precision, str) else int(precision), int(max_iters),
                        float(ru_delta), net.handle if net is not None else None, int(chunk), int(bool(timing)),
                        FORM[formulation] if isinstance(formulation, str) else int(formulation), 0,
                        PRECOND[precond] if isinstance(precond, str) else int(precond), int(debug_breakdown_at),
                        float(stop_margin), DRIVER[driver] if isinstance(driver, str) else int(driver),
                        int(barrier_spins))


def solve(A: Csr, b, x0=None, tol=1e-10, precision="fp64", net=None, max_iters=0, ru_delta=0.0,
          chunk=0, timing=False, x=None, raise_on_error=True, formulation="pinned", precond="none",
          debug_breakdown_at=0, stop_margin=0.0, driver="auto", barrier_spins=0):
    """Solve A x = b on the device.  Returns (x, info dict)."""
    torch = _torch()
    if x is None:
        x = torch.empty(A.n, dtype=torch.float64, device=b.device)
    opts = solve_opts(precision, max_iters, ru_delta, net, chunk, timing, formulation, precond, debug_breakdown_at,
                      stop_margin, driver, barrier_spins)
    info = CfdSolveInfo()
    rc = load().cfd_solve(A.handle, _ptr(b, torch.float64, A.n, "b"), _ptr(x0, torch.float64, A.n, "x0"),
                          float(tol), ctypes.byref(opts), _ptr(x, torch.float64, A.n, "x"),
                          ctypes.byref(info), _stream())
    d = info.as_dict()
    if rc != 0 and raise_on_error:
        check(rc)
    d["rc"] = rc
    return x, d


class State:
    """Cavity state on the MAC grid, device float64 tensors (cfd_state)."""

    def __init__(self, dims, nu=0.0, rho=1.0, lid_u=1.0, g=(0.0, 0.0, 0.0), pin=0, h=None, device="cuda",
                 keep_rhs=False):
        torch = _torch()
        self.grid = make_grid(dims, h)
        nx, ny, nz = self.grid.nx, self.grid.ny, self.grid.nz
        self.dims = (nx, ny, nz)
        self.u = torch.zeros((nx + 1) * ny * nz, dtype=torch.float64, device=device)
        self.v = torch.zeros(nx * (ny + 1) * nz, dtype=torch.float64, device=device)
        self.w = torch.zeros(nx * ny * (nz + 1), dtype=torch.float64, device=device)
        self.p = torch.ones(nx * ny * nz, dtype=torch.float64, device=device)
        self.A = Csr(self.dims, pin, self.grid.h)
        self.rhs = torch.zeros(nx * ny * nz, dtype=torch.float64, device=device) if keep_rhs else None
        self.c = CfdState(self.grid, self.u.data_ptr(), self.v.data_ptr(), self.w.data_ptr(), self.p.data_ptr(),
                          float(nu), float(rho), float(lid_u), float(g[0]), float(g[1]), float(g[2]), 0.0, 0,
                          self.A.handle, self.rhs.data_ptr() if keep_rhs else None)

    @property
    def t(self):
        return self.c.t

    @property
    def step_count(self):
        return self.c.step


def step(S: State, dt, tol=1e-10, precision="fp64", net=None, max_iters=0, ru_delta=0.0, chunk=0,
         formulation="pinned", guess="zero", precond="none", stop_margin=0.0, driver="auto"):
    """One time step (cfd_step).  guess: "zero" (or the network's prediction
    when net is given) or "previous" (start from the pressure in S.p)."""
    opts = solve_opts(precision, max_iters, ru_delta, net, chunk, False, formulation, precond,
                      stop_margin=stop_margin, driver=driver)
    if guess not in ("zero", "previous"):
        raise ValueError("guess must be 'zero' or 'previous'")
    opts.step_guess = 1 if guess == "previous" else 0
    info = CfdSolveInfo()
    check(load().cfd_step(ctypes.byref(S.c), float(dt), float(tol), ctypes.byref(opts), ctypes.byref(info),
                          _stream()))
    return info.as_dict()


class Net:
    """Warm-start network (cfd_net_*)."""

    def __init__(self, init=None, channels=16, layers=4):
        import numpy as np
        lib = load()
        self.channels, self.layers = int(channels), int(layers)
        self.count = int(lib.cfd_net_param_count(self.channels, self.layers))
        self._h = ctypes.c_void_p()
        buf = None
        if init is not None:
            arr = np.ascontiguousarray(init, dtype=np.float32)
            if arr.size != self.count:
                raise ValueError(f"init must have {self.count} values")
            buf = arr.ctypes.data_as(ctypes.c_void_p)
            self._keep = arr
        check(lib.cfd_net_create(self.channels, self.layers, buf, ctypes.byref(self._h)))

    @property
    def handle(self):
        return self._h

    def forward(self, dims, b, y=None, h=None):
        torch = _torch()
        g = make_grid(dims, h)
        n = g.nx * g.ny * g.nz
        if y is None:
            y = torch.empty(n, dtype=torch.float64, device=b.device)
        check(load().cfd_net_forward(self._h, ctypes.byref(g), _ptr(b, torch.float64, n, "b"),
                                     _ptr(y, torch.float64, n, "y"), _stream()))
        return y

    def training_pair(self, dims, b, p, inp=None, target=None):
        """cfd_net_training_pair: (b / rms b, (p - mean p) / rms(p - mean p)) as float32."""
        torch = _torch()
        g = make_grid(dims)
        n = g.nx * g.ny * g.nz
        if inp is None:
            inp = torch.empty(n, dtype=torch.float32, device=b.device)
        if target is None:
            target = torch.empty(n, dtype=torch.float32, device=b.device)
        check(load().cfd_net_training_pair(self._h, ctypes.byref(g), _ptr(b, torch.float64, n, "b"),
                                           _ptr(p, torch.float64, n, "p"), _ptr(inp, torch.float32, n, "input"),
                                           _ptr(target, torch.float32, n, "target"), _stream()))
        return inp, target

    def train_step(self, dims, inp, target, lr, batch=None):
        torch = _torch()
        g = make_grid(dims)
        n = g.nx * g.ny * g.nz
        batch = batch or inp.numel() // n
        loss = ctypes.c_float()
        check(load().cfd_net_train_step(self._h, ctypes.byref(g), int(batch),
                                        _ptr(inp, torch.float32, batch * n, "input"),
                                        _ptr(target, torch.float32, batch * n, "target"), float(lr),
                                        ctypes.byref(loss), _stream()))
        return loss.value

    def gradient(self, dims, inp, target, batch=None):
        import numpy as np
        torch = _torch()
        g = make_grid(dims)
        n = g.nx * g.ny * g.nz
        batch = batch or inp.numel() // n
        grad = np.zeros(self.count, dtype=np.float32)
        loss = ctypes.c_float()
        check(load().cfd_net_gradient(self._h, ctypes.byref(g), int(batch),
                                      _ptr(inp, torch.float32, batch * n, "input"),
                                      _ptr(target, torch.float32, batch * n, "target"),
                                      grad.ctypes.data_as(ctypes.c_void_p), ctypes.byref(loss), _stream()))
        return loss.value, grad

    def params(self):
        import numpy as np
        out = np.zeros(self.count, dtype=np.float32)
        check(load().cfd_net_get_params(self._h, out.ctypes.data_as(ctypes.c_void_p), self.count))
        return out

    def set_params(self, theta):
        import numpy as np
        arr = np.ascontiguousarray(theta, dtype=np.float32)
        check(load().cfd_net_set_params(self._h, arr.ctypes.data_as(ctypes.c_void_p), arr.size))

    def close(self):
        if self._h:
            load().cfd_net_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def conv3d_forward(dims, cin, cout, x_bits, w_bits, relu=False):
    """One convolution layer on bf16 bit patterns (int16 tensors); float32 output."""
    torch = _torch()
    g = make_grid(dims)
    n = g.nx * g.ny * g.nz
    y = torch.empty(n * cout, dtype=torch.float32, device=x_bits.device)
    check(load().cfd_conv3d_forward(ctypes.byref(g), cin, cout, _ptr(x_bits, torch.int16, n * cin, "x"),
                                    _ptr(w_bits, torch.int16, 27 * cin * cout, "w"),
                                    _ptr(y, torch.float32, n * cout, "y"), int(bool(relu)), _stream()))
    return y


def conv3d_backward_data(dims, cin, cout, dy_bits, w_bits):
    torch = _torch()
    g = make_grid(dims)
    n = g.nx * g.ny * g.nz
    dx = torch.empty(n * cin, dtype=torch.float32, device=dy_bits.device)
    check(load().cfd_conv3d_backward_data(ctypes.byref(g), cin, cout, _ptr(dy_bits, torch.int16, n * cout, "dy"),
                                          _ptr(w_bits, torch.int16, 27 * cin * cout, "w"),
                                          _ptr(dx, torch.float32, n * cin, "dx"), _stream()))
    return dx


def conv3d_backward_weight(dims, cin, cout, x_bits, dy_bits):
    torch = _torch()
    g = make_grid(dims)
    n = g.nx * g.ny * g.nz
    dw = torch.empty(27 * cin * cout, dtype=torch.float32, device=x_bits.device)
    check(load().cfd_conv3d_backward_weight(ctypes.byref(g), cin, cout, _ptr(x_bits, torch.int16, n * cin, "x"),
                                            _ptr(dy_bits, torch.int16, n * cout, "dy"),
                                            _ptr(dw, torch.float32, 27 * cin * cout, "dw"), _stream()))
    return dw
