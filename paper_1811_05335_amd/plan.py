"""Python binding of the C ABI: argument marshalling only.  Every step of the transforms runs
in the HIP library; torch supplies device memory and the stream."""
from __future__ import annotations

import ctypes as C

import torch

from . import _lib
from ._lib import Options, Status, check, load


def _stream_handle() -> int:
    return torch.cuda.current_stream().cuda_stream


def _ptr(t: torch.Tensor) -> int:
    return t.data_ptr()


class NfftPlan:
    """A plan of the direct inverse NFFT for fixed nodes (see include/infft.h).

    M          coefficients per dimension (even), tuple of length d in {1, 2}
    x          nodes, float64 tensor (N, d) on the GPU (wrapped onto the torus by the library)
    sigma, m   oversampling factor and window cut-off
    precision  "f32" (complex64 data, FP32 spreading/FFT) or "f64" (complex128)
    rho        ridge of the local least-squares problems of the B optimisation
    kernel     kernel of the inverse: "window" (the NFFT's window) or "dirichlet" (Remark 3.19)
    work_slots sets of transform work buffers; `set_slot` picks one, so that transforms on different
               slots and streams may overlap
    workspace  True: the plan lives in one torch-allocated device buffer (nfft_plan_ws), and no call
               on it allocates device memory; large_mib and ansatz1 size its parts for large local
               problems and for Algorithm 3.10
    """

    def __init__(self, M, x: torch.Tensor, sigma: float = 2.0, m: int = 4, precision: str = "f64",
                 rho: float = 1e-8, max_rhs: int = 1, tile=None, kernel: str = "window",
                 work_slots: int = 1, workspace: bool = False, large_mib: int = 0, ansatz1: bool = False):
        lib = load()
        self.M = tuple(int(v) for v in (M if isinstance(M, (tuple, list)) else (M,)))
        self.d = len(self.M)
        x = self._nodes(x)
        self.N = x.shape[0]
        self.sigma, self.m = float(sigma), int(m)
        self.precision = precision
        self.ctype = torch.complex64 if precision == "f32" else torch.complex128
        self.taps = (2 * self.m + 1) ** self.d
        o = Options()
        lib.infft_default_options(C.byref(o))
        o.precision = _lib.INFFT_F32 if precision == "f32" else _lib.INFFT_F64
        o.max_rhs = int(max_rhs)
        o.rho = float(rho)
        o.inverse_kernel = _lib.KERNELS[kernel]
        o.work_slots = int(work_slots)
        if tile is not None:
            for t, v in enumerate(tile):
                o.tile[t] = int(v)
        Ms = (C.c_int64 * self.d)(*self.M)
        h = C.c_void_p()
        self._ws = None
        if workspace:
            o.large_mib = int(large_mib)
            o.ansatz1 = int(bool(ansatz1))
            nb = C.c_size_t()
            check(lib.nfft_plan_workspace_bytes(self.d, Ms, self.N, self.sigma, self.m, C.byref(o), C.byref(nb)))
            self._ws = torch.empty(int(nb.value), dtype=torch.uint8, device=x.device)
            check(lib.nfft_plan_ws(C.byref(h), self.d, Ms, self.N, self.sigma, self.m, C.c_void_p(_ptr(x)),
                                   C.byref(o), C.c_void_p(_ptr(self._ws)), nb, C.c_void_p(_stream_handle())))
        else:
            check(lib.nfft_plan(C.byref(h), self.d, Ms, self.N, self.sigma, self.m, C.c_void_p(_ptr(x)),
                                C.byref(o), C.c_void_p(_stream_handle())))
        self._h = h
        self._x = x
        self.device = x.device
        # node-set version: bumped by set_nodes; B_opt records the version it was computed for
        self.nodes_version = 0
        self.bopt_version = -1

    # -------------------------------------------------------------- helpers
    def _nodes(self, x: torch.Tensor) -> torch.Tensor:
        if not x.is_cuda or x.dtype != torch.float64:
            raise TypeError("x must be a float64 CUDA tensor")
        if x.dim() == 1:
            x = x[:, None]
        if x.shape[1] != self.d:
            raise ValueError(f"x must have shape (N, {self.d})")
        return x.contiguous()

    def _sync_stream(self):
        check(load().nfft_set_stream(self._h, C.c_void_p(_stream_handle())))

    def _coeffs(self, a: torch.Tensor):
        if a.dtype != self.ctype or not a.is_cuda:
            raise TypeError(f"expected a {self.ctype} CUDA tensor")
        if tuple(a.shape[-self.d:]) != self.M:
            raise ValueError(f"trailing shape must be {self.M}")
        lead = a.shape[: a.dim() - self.d]
        R = 1
        for v in lead:
            R *= int(v)
        return a.contiguous(), lead, R

    def _samples(self, a: torch.Tensor):
        if a.dtype != self.ctype or not a.is_cuda:
            raise TypeError(f"expected a {self.ctype} CUDA tensor")
        if a.shape[-1] != self.N:
            raise ValueError(f"last dimension must be N = {self.N}")
        lead = a.shape[:-1]
        R = 1
        for v in lead:
            R *= int(v)
        return a.contiguous(), lead, R

    # -------------------------------------------------------------- entry points
    def set_nodes(self, x: torch.Tensor) -> None:
        x = self._nodes(x)
        if x.shape[0] != self.N:
            raise ValueError("set_nodes keeps N fixed")
        self._sync_stream()
        check(load().nfft_set_nodes(self._h, C.c_void_p(_ptr(x))))
        self._x = x
        self.nodes_version += 1

    def trafo(self, fhat: torch.Tensor) -> torch.Tensor:
        fh, lead, R = self._coeffs(fhat)
        out = torch.empty(tuple(lead) + (self.N,), dtype=self.ctype, device=self.device)
        self._sync_stream()
        check(load().nfft_trafo(self._h, C.c_void_p(_ptr(fh)), C.c_void_p(_ptr(out)), R))
        # which trafo the current slot's grid may hold (read by the autograd backward)
        self._trafo_seq = getattr(self, "_trafo_seq", 0) + 1
        return out

    def adjoint(self, f: torch.Tensor) -> torch.Tensor:
        ff, lead, R = self._samples(f)
        out = torch.empty(tuple(lead) + self.M, dtype=self.ctype, device=self.device)
        self._sync_stream()
        check(load().nfft_adjoint(self._h, C.c_void_p(_ptr(ff)), C.c_void_p(_ptr(out)), R))
        return out

    def set_slot(self, slot: int) -> None:
        """Work-buffer set of the following transforms (calls on different slots and streams may
        overlap on the device)."""
        check(load().nfft_set_slot(self._h, int(slot)))
        self._slot = int(slot)

    def precompute_B(self) -> None:
        self._sync_stream()
        check(load().infft_precompute_B(self._h))
        self.bopt_version = self.nodes_version

    def precompute_Bstar(self) -> None:
        """Algorithm 3.10 (ansatz 1): per-node optimisation of B^*; afterwards `apply` is the
        estimate (1/M) D^* F^* B_opt^* f and `apply_adjoint` the inverse adjoint of Remark 3.15."""
        self._sync_stream()
        check(load().infft_precompute_Bstar(self._h))
        self.bopt_version = self.nodes_version

    def apply(self, f: torch.Tensor) -> torch.Tensor:
        ff, lead, R = self._samples(f)
        out = torch.empty(tuple(lead) + self.M, dtype=self.ctype, device=self.device)
        self._sync_stream()
        check(load().infft_apply(self._h, C.c_void_p(_ptr(ff)), C.c_void_p(_ptr(out)), R))
        return out

    def apply_adjoint(self, h: torch.Tensor) -> torch.Tensor:
        hh, lead, R = self._coeffs(h)
        out = torch.empty(tuple(lead) + (self.N,), dtype=self.ctype, device=self.device)
        self._sync_stream()
        check(load().infft_apply_adjoint(self._h, C.c_void_p(_ptr(hh)), C.c_void_p(_ptr(out)), R))
        return out

    def grad_x(self, fhat: torch.Tensor, gradf: torch.Tensor) -> torch.Tensor:
        fh, lead, R = self._coeffs(fhat)
        gf, lead2, R2 = self._samples(gradf)
        if R2 != R:
            raise ValueError("fhat and gradf need the same number of right-hand sides")
        out = torch.empty((self.N, self.d), dtype=torch.float64, device=self.device)
        self._sync_stream()
        check(load().nfft_grad_x(self._h, C.c_void_p(_ptr(fh)), C.c_void_p(_ptr(gf)), C.c_void_p(_ptr(out)), R))
        return out

    def grad_x_after_trafo(self, gradf: torch.Tensor) -> torch.Tensor:
        """The node gradient of grad_x, from the grid the last trafo on the current work slot left
        (no FFT of fhat); the library raises if another call has written that grid since."""
        gf, lead, R = self._samples(gradf)
        out = torch.empty((self.N, self.d), dtype=torch.float64, device=self.device)
        self._sync_stream()
        check(load().nfft_grad_x_after_trafo(self._h, C.c_void_p(_ptr(gf)), C.c_void_p(_ptr(out)), R))
        return out

    def grad_x_bopt(self, f: torch.Tensor, gradfc: torch.Tensor) -> torch.Tensor:
        """Node gradient through B_opt(x) of a loss of fcheck = apply(f), f held fixed."""
        ff, lead, R = self._samples(f)
        gc, lead2, R2 = self._coeffs(gradfc)
        if R2 != R:
            raise ValueError("f and gradfc need the same number of right-hand sides")
        out = torch.empty((self.N, self.d), dtype=torch.float64, device=self.device)
        self._sync_stream()
        check(load().infft_grad_x_bopt(self._h, C.c_void_p(_ptr(ff)), C.c_void_p(_ptr(gc)),
                                       C.c_void_p(_ptr(out)), R))
        return out

    def get_B(self) -> torch.Tensor:
        out = torch.empty((self.N, self.taps), dtype=torch.complex128, device=self.device)
        self._sync_stream()
        check(load().infft_get_B(self._h, C.c_void_p(_ptr(out))))
        return out

    def export_B(self) -> bytes:
        """B_opt with the parameters and nodes it belongs to, serialised (infft_plan_export)."""
        lib = load()
        nb = C.c_size_t()
        check(lib.infft_plan_export(self._h, None, C.byref(nb)))
        buf = C.create_string_buffer(int(nb.value))
        self._sync_stream()
        check(lib.infft_plan_export(self._h, buf, C.byref(nb)))
        return buf.raw[: int(nb.value)]

    def import_B(self, data: bytes) -> None:
        """Loads an exported B_opt (and its nodes) into this plan (infft_plan_import)."""
        self._sync_stream()
        buf = C.create_string_buffer(bytes(data), len(data))
        check(load().infft_plan_import(self._h, buf, len(data)))
        # the plan's nodes are now the exported ones (they follow the 72-byte header)
        import numpy as np
        nd = self.N * self.d
        self._x = torch.from_numpy(np.frombuffer(data, dtype=np.float64, count=nd, offset=72).copy()).reshape(
            self.N, self.d).to(self.device)
        self.nodes_version += 1
        self.bopt_version = self.nodes_version

    def status(self) -> dict:
        st = Status()
        code = load().nfft_plan_status(self._h, C.byref(st))
        d = {name: getattr(st, name) for name, _ in Status._fields_}
        d["code"] = code
        return d

    def profile_begin(self, kernel_class: str) -> None:
        """Time every launch of one kernel class with HIP events on the plan's stream."""
        self._sync_stream()
        check(load().infft_profile_begin(self._h, _lib.KERNEL_CLASSES[kernel_class]))

    def profile_end(self):
        """(summed milliseconds, number of launches) since profile_begin."""
        ms = C.c_double()
        n = C.c_int64()
        check(load().infft_profile_end(self._h, C.byref(ms), C.byref(n)))
        return ms.value, n.value

    def autotune(self, reps: int = 10) -> dict:
        """Times each FFT direction in a HIP graph with the default shapes and with 1..16
        sub-transforms per workgroup per pass, and keeps the fastest; returns the choice per
        direction and step (0: the default), and the spreading's right-hand sides per pass
        (`spread_rhs`, tuned when max_rhs > 1)."""
        self._sync_stream()
        check(load().infft_autotune(self._h, int(reps)))
        lib = load()
        out = {f"{'to_grid' if d == 0 else 'to_coeff'}_{k}": lib.infft_autotune_rows(self._h, d, k)
               for d in (0, 1) for k in (0, 1)}
        out["spread_rhs"] = lib.infft_autotune_rhs_chunk(self._h)
        return out

    def device_bytes(self) -> int:
        return int(load().nfft_plan_device_bytes(self._h))

    def close(self) -> None:
        if getattr(self, "_h", None):
            load().nfft_plan_destroy(self._h)
            self._h = None
        self._ws = None   # a workspace plan's memory, released after the plan

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class NfftBatchPlan(NfftPlan):
    """Many independent one-dimensional problems of uneven sizes in one plan (nfft_plan_batched):
    every stage runs for all problems in one kernel launch.

    Ms, Ns     coefficients (even) and nodes of each problem
    x          float64 CUDA tensor with the nodes of all problems one after the other
    Data are flat, problem-major tensors: coefficients [problem][R][M_i] (length R * sum Ms),
    samples [problem][R][N_i] (length R * sum Ns), with R <= max_rhs given to each call;
    `pack` and `unpack` convert from and to lists of per-problem (R, M_i) / (R, N_i) tensors.
    """

    def __init__(self, Ms, Ns, x: torch.Tensor, sigma: float = 2.0, m: int = 4, precision: str = "f64",
                 rho: float = 1e-8, max_rhs: int = 1, kernel: str = "window"):
        lib = load()
        self.Ms = [int(v) for v in Ms]
        self.Ns = [int(v) for v in Ns]
        if len(self.Ms) != len(self.Ns) or not self.Ms:
            raise ValueError("Ms and Ns must be non-empty and of equal length")
        self.d = 1
        self.M = (sum(self.Ms),)
        self.N = sum(self.Ns)
        x = self._nodes(x)
        if x.shape[0] != self.N:
            raise ValueError("x must hold sum(Ns) nodes")
        self.sigma, self.m = float(sigma), int(m)
        self.precision = precision
        self.ctype = torch.complex64 if precision == "f32" else torch.complex128
        self.taps = 2 * self.m + 1
        self.max_rhs = int(max_rhs)
        o = Options()
        lib.infft_default_options(C.byref(o))
        o.precision = _lib.INFFT_F32 if precision == "f32" else _lib.INFFT_F64
        o.max_rhs = self.max_rhs
        o.rho = float(rho)
        o.inverse_kernel = _lib.KERNELS[kernel]
        n = len(self.Ms)
        Mv = (C.c_int64 * n)(*self.Ms)
        Nv = (C.c_int64 * n)(*self.Ns)
        h = C.c_void_p()
        check(lib.nfft_plan_batched(C.byref(h), n, Mv, Nv, self.sigma, self.m, C.c_void_p(_ptr(x)), C.byref(o),
                                    C.c_void_p(_stream_handle())))
        self._h = h
        self._x = x
        self.device = x.device
        self.nodes_version = 0
        self.bopt_version = -1

    def _flat(self, a: torch.Tensor, per: int):
        if a.dtype != self.ctype or not a.is_cuda:
            raise TypeError(f"expected a {self.ctype} CUDA tensor")
        a = a.reshape(-1).contiguous()
        if a.numel() % per:
            raise ValueError(f"length must be a multiple of {per}")
        R = a.numel() // per
        if R < 1 or R > self.max_rhs:
            raise ValueError(f"1 <= R <= max_rhs = {self.max_rhs}")
        return a, R

    def _coeffs(self, a):
        a, R = self._flat(a, self.M[0])
        return a, (R * self.M[0],), R

    def _samples(self, a):
        a, R = self._flat(a, self.N)
        return a, (R * self.N,), R

    def _out(self, n):
        return torch.empty(n, dtype=self.ctype, device=self.device)

    def trafo(self, fhat):
        fh, _, R = self._coeffs(fhat)
        out = self._out(R * self.N)
        self._sync_stream()
        check(load().nfft_trafo(self._h, C.c_void_p(_ptr(fh)), C.c_void_p(_ptr(out)), R))
        return out

    def adjoint(self, f):
        ff, _, R = self._samples(f)
        out = self._out(R * self.M[0])
        self._sync_stream()
        check(load().nfft_adjoint(self._h, C.c_void_p(_ptr(ff)), C.c_void_p(_ptr(out)), R))
        return out

    def apply(self, f):
        ff, _, R = self._samples(f)
        out = self._out(R * self.M[0])
        self._sync_stream()
        check(load().infft_apply(self._h, C.c_void_p(_ptr(ff)), C.c_void_p(_ptr(out)), R))
        return out

    def apply_adjoint(self, h):
        hh, _, R = self._coeffs(h)
        out = self._out(R * self.N)
        self._sync_stream()
        check(load().infft_apply_adjoint(self._h, C.c_void_p(_ptr(hh)), C.c_void_p(_ptr(out)), R))
        return out

    def grad_x(self, fhat, gradf):
        fh, _, R = self._coeffs(fhat)
        gf, _, R2 = self._samples(gradf)
        if R2 != R:
            raise ValueError("fhat and gradf need the same number of right-hand sides")
        out = torch.empty((self.N, 1), dtype=torch.float64, device=self.device)
        self._sync_stream()
        check(load().nfft_grad_x(self._h, C.c_void_p(_ptr(fh)), C.c_void_p(_ptr(gf)), C.c_void_p(_ptr(out)), R))
        return out

    def pack(self, arrays, kind: str) -> torch.Tensor:
        """Per-problem tensors of shape (R, M_i) ("coeffs") or (R, N_i) ("samples") -> flat tensor."""
        return torch.cat([a.reshape(-1) for a in arrays]).contiguous()

    def unpack(self, flat: torch.Tensor, kind: str, R: int):
        sizes = self.Ms if kind == "coeffs" else self.Ns
        out, o = [], 0
        for n in sizes:
            out.append(flat[o:o + R * n].reshape(R, n))
            o += R * n
        return out


# Function names of the C ABI, for callers who prefer them to the class.
def nfft_plan_batched(Ms, Ns, x, sigma=2.0, m=4, **kw) -> NfftBatchPlan:
    return NfftBatchPlan(Ms, Ns, x, sigma=sigma, m=m, **kw)


def nfft_plan(M, x, sigma=2.0, m=4, **kw) -> NfftPlan:
    return NfftPlan(M, x, sigma, m, **kw)


def nfft_set_nodes(plan: NfftPlan, x):
    return plan.set_nodes(x)


def nfft_trafo(plan: NfftPlan, fhat):
    return plan.trafo(fhat)


def nfft_adjoint(plan: NfftPlan, f):
    return plan.adjoint(f)


def infft_precompute_B(plan: NfftPlan):
    return plan.precompute_B()


def infft_precompute_Bstar(plan: NfftPlan):
    return plan.precompute_Bstar()


def infft_apply(plan: NfftPlan, f):
    return plan.apply(f)


def infft_apply_adjoint(plan: NfftPlan, h):
    return plan.apply_adjoint(h)


def nfft_grad_x(plan: NfftPlan, fhat, gradf):
    return plan.grad_x(fhat, gradf)


def infft_get_B(plan: NfftPlan):
    return plan.get_B()


def nfft_plan_status(plan: NfftPlan):
    return plan.status()


def nfft_plan_destroy(plan: NfftPlan):
    plan.close()
