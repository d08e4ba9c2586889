"""Python front end of the DBFFT HIP library.

PyTorch provides device memory and the stream; all arithmetic runs in
libdbfft.so.  Shapes follow include/dbfft.h: real fields (c, n1, n2, n3)
float64, Fourier unknowns (3, n1, n2, n3//2+1) complex128, 3x3 host arrays.
"""
from __future__ import annotations

import ctypes as ct

import numpy as np
import torch

from . import _native as nat

_KIN = {"small": nat.SMALL, "finite": nat.FINITE}
_PREC = {"fp64": nat.FP64, "fp32_mixed": nat.FP32_MIXED}
_MAT = {
    "iso_phase": (nat.MAT_ISO_PHASE, torch.uint8),
    "iso_field": (nat.MAT_ISO_FIELD, torch.float64),
    "aniso_grain": (nat.MAT_ANISO_GRAIN, torch.int32),
    "j2vp_cubic": (nat.MAT_J2VP_CUBIC, torch.int32),
    "neohooke": (nat.MAT_NEOHOOKE, torch.uint8),
    "svk": (nat.MAT_SVK, torch.uint8),
}


def _ptr(t):
    return ct.c_void_p(t.data_ptr())


def _info_dict(info):
    return {
        "pcg_iters": info.pcg_iters,
        "newton_iters": info.newton_iters,
        "increments": info.increments,
        "refine_steps": info.refine_steps,
        "status": info.status,
        "eq_res": info.eq_res,
        "load_res": info.load_res,
        "sigma_bar": np.array(info.sigma_bar[:]).reshape(3, 3),
        "eps_bar": np.array(info.eps_bar[:]).reshape(3, 3),
    }


def apply_noalloc(n, material, field, params, u, out, stream=None):
    """dbfft_apply_noalloc: the FP64 small-strain operator of Cell.apply for
    an "iso_phase" or "iso_field" material, with no context and no device
    allocation by the library (its workspace is a static device array).
    `field`, `u` and `out` must already be contiguous device tensors of the
    right dtype (uint8 or float64 field; float64 (3, n1, n2, n3) u and out).
    Asynchronous: `out` is ready when `stream` (default: the current one)
    has run the work."""
    kind, dtype = _MAT[material]
    if material not in ("iso_phase", "iso_field"):
        raise ValueError("apply_noalloc takes iso_phase or iso_field materials")
    n = tuple(int(v) for v in n)
    for t, dt in ((field, dtype), (u, torch.float64), (out, torch.float64)):
        if not (t.is_cuda and t.dtype == dt and t.is_contiguous()):
            raise ValueError("field, u and out must be contiguous device tensors of the documented dtypes")
    if field.numel() != int(np.prod(n)) or u.shape != (3,) + n or out.shape != (3,) + n:
        raise ValueError("shapes do not match the grid")
    if stream is None:
        stream = torch.cuda.current_stream(u.device)
    p = np.ascontiguousarray(np.asarray(params, dtype=np.float64).reshape(-1))
    dims = (ct.c_int64 * 3)(*n)
    nat.check(nat.lib().dbfft_apply_noalloc(dims, kind, _ptr(field), p.ctypes.data_as(ct.POINTER(ct.c_double)),
                                            int(p.size), _ptr(u), _ptr(out), ct.c_void_p(stream.cuda_stream)))
    return out


class Cell:
    """One periodic cell (grid + material) bound to a HIP stream."""

    def __init__(self, n, material, field, params, kinematics="small", precision="fp64", stream=None,
                 device="cuda", lengths=None):
        self.n = tuple(int(v) for v in n)
        self.N = int(np.prod(self.n))
        self.kin = kinematics
        self.prec = precision
        self.material = material
        kind, dtype = _MAT[material]
        f = torch.as_tensor(field).to(device=device, dtype=dtype).contiguous()
        if f.numel() != self.N:
            raise ValueError("material field must have n1*n2*n3 entries")
        self.field = f
        self.device = f.device
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        p = np.ascontiguousarray(np.asarray(params, dtype=np.float64).reshape(-1))
        dims = (ct.c_int64 * 3)(*self.n)
        h = ct.c_void_p()
        nat.check(nat.lib().dbfft_setup(ct.byref(h), dims, _KIN[kinematics], _PREC[precision], kind,
                                        _ptr(f), p.ctypes.data_as(ct.POINTER(ct.c_double)), int(p.size),
                                        ct.c_void_p(stream.cuda_stream)))
        self._h = h
        self.ncomp = 6 if kinematics == "small" else 9
        self.half = (self.n[0], self.n[1], self.n[2] // 2 + 1)
        self.lengths = (1.0, 1.0, 1.0)
        if lengths is not None:
            self.set_lengths(lengths)

    def set_lengths(self, lengths):
        """dbfft_set_lengths: side lengths L1, L2, L3 of the cell."""
        L = [float(v) for v in lengths]
        if len(L) != 3:
            raise ValueError("three cell lengths expected")
        nat.check(nat.lib().dbfft_set_lengths(self._h, nat.dvec(L, 3)))
        self.lengths = tuple(L)

    def close(self):
        if getattr(self, "_h", None):
            nat.lib().dbfft_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # ------------------------------------------------------------------
    def solve(self, load, stress_mask=None, n_increments=1, dt=1.0, raise_on_fail=True, **opts):
        load = np.asarray(load, dtype=np.float64).reshape(9)
        mask = np.zeros(9, dtype=np.uint8) if stress_mask is None else \
            np.asarray(stress_mask, dtype=bool).reshape(9).astype(np.uint8)
        o = nat.default_opts(**opts)
        info = nat.Info()
        st = nat.lib().dbfft_solve(self._h, nat.dvec(load), (ct.c_uint8 * 9)(*mask.tolist()), int(n_increments),
                                   float(dt), ct.byref(o), ct.byref(info))
        if st != nat.DBFFT_OK and raise_on_fail:
            nat.check(st)
        d = _info_dict(info)
        d["status"] = st
        return d

    def apply(self, u):
        u = u.to(device=self.device, dtype=torch.float64).contiguous()
        f = torch.empty_like(u)
        nat.check(nat.lib().dbfft_apply(self._h, _ptr(u), _ptr(f)))
        return f

    def apply_fourier(self, a, e_macro=None):
        a = a.to(device=self.device, dtype=torch.complex128).contiguous()
        f = torch.empty_like(a)
        sig = (ct.c_double * 9)()
        em = None if e_macro is None else nat.dvec(np.asarray(e_macro, dtype=np.float64).reshape(9))
        nat.check(nat.lib().dbfft_apply_fourier(self._h, _ptr(a), em, _ptr(f), sig))
        return f, np.array(sig[:]).reshape(3, 3)

    def solve_many(self, loads, stress_mask=None, nstreams=2, raise_on_fail=True, **opts):
        """dbfft_solve_many: the loads (a list of 3x3) solved as independent
        PCG solves on `nstreams` concurrent streams.  Returns the list of
        info dicts (one per load)."""
        L = np.ascontiguousarray(np.asarray(loads, dtype=np.float64).reshape(-1, 9))
        s = L.shape[0]
        mask = np.zeros(9, dtype=np.uint8) if stress_mask is None else \
            np.asarray(stress_mask, dtype=bool).reshape(9).astype(np.uint8)
        o = nat.default_opts(**opts)
        infos = (nat.Info * s)()
        st = nat.lib().dbfft_solve_many(self._h, s, L.ctypes.data_as(ct.POINTER(ct.c_double)),
                                        (ct.c_uint8 * 9)(*mask.tolist()), ct.byref(o), infos, int(nstreams))
        if st != nat.DBFFT_OK and raise_on_fail:
            nat.check(st)
        return [_info_dict(infos[j]) for j in range(s)]

    def solve_block(self, loads, stress_mask=None, raise_on_fail=True, **opts):
        """dbfft_solve_block: the loads (a list of 3x3) solved together by
        block PCG.  Returns (list of info dicts, operator applications)."""
        L = np.ascontiguousarray(np.asarray(loads, dtype=np.float64).reshape(-1, 9))
        s = L.shape[0]
        mask = np.zeros(9, dtype=np.uint8) if stress_mask is None else \
            np.asarray(stress_mask, dtype=bool).reshape(9).astype(np.uint8)
        o = nat.default_opts(**opts)
        infos = (nat.Info * s)()
        applies = ct.c_int32()
        st = nat.lib().dbfft_solve_block(self._h, s, L.ctypes.data_as(ct.POINTER(ct.c_double)),
                                         (ct.c_uint8 * 9)(*mask.tolist()), ct.byref(o), infos, ct.byref(applies))
        if st != nat.DBFFT_OK and raise_on_fail:
            nat.check(st)
        out = [_info_dict(infos[j]) for j in range(s)]
        return out, applies.value

    def homogenize(self, strain=False, stress=False, displacement=False):
        sig = (ct.c_double * 9)()
        eps = (ct.c_double * 9)()
        out = {}
        fs = torch.empty((self.ncomp,) + self.n, dtype=torch.float64, device=self.device) if strain else None
        fp = torch.empty((self.ncomp,) + self.n, dtype=torch.float64, device=self.device) if stress else None
        fu = torch.empty((3,) + self.n, dtype=torch.float64, device=self.device) if displacement else None
        nat.check(nat.lib().dbfft_homogenize(self._h, sig, eps, _ptr(fs) if fs is not None else None,
                                             _ptr(fp) if fp is not None else None,
                                             _ptr(fu) if fu is not None else None))
        out["sigma_bar"] = np.array(sig[:]).reshape(3, 3)
        out["eps_bar"] = np.array(eps[:]).reshape(3, 3)
        if strain:
            out["strain"] = fs
        if stress:
            out["stress"] = fp
        if displacement:
            out["displacement"] = fu
        return out

    def residuals(self, strain=None, stress=None, load=None, stress_mask=None):
        """dbfft_residuals: (equilibrium, compatibility, loading strain part,
        loading stress part) of the given real fields, or of the last
        solve's fields where a field is None."""
        def field(t):
            if t is None:
                return None, None
            t = t.to(device=self.device, dtype=torch.float64).contiguous()
            if tuple(t.shape) != (self.ncomp,) + tuple(self.n):
                raise ValueError(f"field of shape {tuple(t.shape)}, expected {(self.ncomp,) + tuple(self.n)}")
            return t, _ptr(t)
        fs, ps = field(strain)
        fp, pp = field(stress)
        ld = None if load is None else nat.dvec(np.asarray(load, dtype=np.float64).reshape(9))
        mk = None if stress_mask is None else \
            (ct.c_uint8 * 9)(*np.asarray(stress_mask, dtype=bool).reshape(9).astype(np.uint8).tolist())
        out = (ct.c_double * 4)()
        nat.check(nat.lib().dbfft_residuals(self._h, ps, pp, ld, mk, out))
        del fs, fp
        return np.array(out[:])

    def solution(self):
        a = torch.empty((3,) + self.half, dtype=torch.complex128, device=self.device)
        e = (ct.c_double * 9)()
        nat.check(nat.lib().dbfft_get_solution(self._h, _ptr(a), e))
        return a, np.array(e[:]).reshape(3, 3)

    def kernel_timing(self, enable):
        """Returns {kind: (total_ms, launches)} accumulated so far, then
        switches event timing on (enable=True, counters reset) or off."""
        ms = (ct.c_double * 16)()
        n = (ct.c_int64 * 16)()
        nat.check(nat.lib().dbfft_kernel_timing(self._h, 1 if enable else 0, ms, n))
        return {k: (ms[i], n[i]) for i, k in enumerate(nat.KERNEL_KINDS)}

    def adjoint(self, G, H=None):
        G = np.asarray(G, dtype=np.float64).reshape(9)
        H = np.zeros(9) if H is None else np.asarray(H, dtype=np.float64).reshape(9)
        grad = torch.empty(self.n, dtype=torch.float64, device=self.device)
        J = ct.c_double()
        nat.check(nat.lib().dbfft_adjoint(self._h, nat.dvec(G), nat.dvec(H), _ptr(grad), ct.byref(J)))
        return grad, J.value


class Batch:
    """Several cells (of one precision, kinematics and material class)
    solved together: one launch per pass over every cell, a captured HIP
    graph per chunk of PCG iterations.  The cells must outlive the batch."""

    def __init__(self, cells, use_graph=True):
        self.cells = list(cells)
        if not self.cells:
            raise ValueError("empty batch")
        for c in self.cells:
            torch.cuda.current_stream(c.device).synchronize()
            c.stream.synchronize()
        arr = (ct.c_void_p * len(self.cells))(*[c._h.value for c in self.cells])
        h = ct.c_void_p()
        nat.check(nat.lib().dbfft_batch_create(ct.byref(h), arr, len(self.cells), 1 if use_graph else 0))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            nat.lib().dbfft_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def tiles(self):
        t = (ct.c_int32 * (3 * len(self.cells)))()
        nat.check(nat.lib().dbfft_batch_tiles(self._h, t))
        return np.array(t[:], dtype=np.int32).reshape(-1, 3)

    def solve(self, loads, stress_masks=None, n_increments=1, dt=1.0, raise_on_fail=True, **opts):
        n = len(self.cells)
        loads = np.ascontiguousarray(np.broadcast_to(np.asarray(loads, dtype=np.float64).reshape(-1, 9), (n, 9)))
        if stress_masks is None:
            masks = np.zeros((n, 9), dtype=np.uint8)
        else:
            masks = np.ascontiguousarray(
                np.broadcast_to(np.asarray(stress_masks, dtype=bool).reshape(-1, 9), (n, 9)).astype(np.uint8))
        o = nat.default_opts(**opts)
        infos = (nat.Info * n)()
        st = nat.lib().dbfft_batch_solve(self._h, loads.ctypes.data_as(ct.POINTER(ct.c_double)),
                                         masks.ctypes.data_as(ct.POINTER(ct.c_uint8)), int(n_increments), float(dt),
                                         ct.byref(o), infos)
        if st != nat.DBFFT_OK and raise_on_fail:
            nat.check(st)
        return [_info_dict(infos[i]) for i in range(n)]


class HomogenizedResponse(torch.autograd.Function):
    """J(E) = G:<sigma> + H:<eps> of a linear cell with per-voxel Young's
    modulus E (Poisson ratio nu), load / stress_mask as in Cell.solve.
    backward runs the adjoint solve of the same operator."""

    @staticmethod
    def forward(ctx, E, load, stress_mask, G, H, nu, precision, tol):
        cell = Cell(E.shape, "iso_field", E.detach(), [nu], precision=precision, device=E.device)
        try:
            cell.solve(load, stress_mask, tol=tol, tol_load=tol)
            h = cell.homogenize()
        except Exception:
            cell.close()
            raise
        J = float(np.sum(np.asarray(G) * h["sigma_bar"]) + np.sum(np.asarray(H) * h["eps_bar"]))
        if ctx.needs_input_grad[0]:
            # the adjoint solve runs in backward, on this cell's solution
            ctx.cell, ctx.G, ctx.H = cell, G, H
        else:
            cell.close()
        return torch.tensor(J, dtype=torch.float64, device=E.device)

    @staticmethod
    def backward(ctx, gout):
        cell = ctx.cell
        try:
            grad, _ = cell.adjoint(ctx.G, ctx.H)
        finally:
            cell.close()
            ctx.cell = None
        return gout * grad, None, None, None, None, None, None, None


def homogenized_response(E, load, stress_mask=None, G=None, H=None, nu=0.3, precision="fp64", tol=1e-10):
    if G is None:
        G = np.zeros((3, 3))
    if H is None:
        H = np.zeros((3, 3))
    return HomogenizedResponse.apply(E, load, stress_mask, G, H, nu, precision, tol)
