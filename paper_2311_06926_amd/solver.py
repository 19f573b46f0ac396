"""Python front end of the MI355X hyper-power Stokes solver.

``Solver`` owns one library context (``hp_setup``) and exposes the C-ABI
calls with the same names on torch tensors that live on the GPU.  torch
provides device memory and the stream only; every operation is a call into
``libhyperpower.so``.
"""
import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import check, hp_opts, hp_solve_info


def _ptr(t):
    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch tensor")
    if t.device.type != "cuda" or t.dtype != torch.float64 or not t.is_contiguous():
        raise ValueError("vectors must be contiguous float64 CUDA tensors")
    return ctypes.c_void_p(t.data_ptr())


class Solver:
    """Context for E^3 elements, velocity degree p, viscosity nu.

    Options (see include/hyperpower.h): c_pen, schur ('Pcq1'|'Pcq2'|'Pcq_pcg'),
    schedule ('literal'|'prev'), precision ('fp64'|'fp32'|'bf16x3'),
    krylov ('minres'|'fgmres'), restart, maxit, order, iters, max_rhs,
    schur_level (eq. Pcq2: the fixed P_{V,l} in B' P_{V,l}^{-1} B; Pcq_pcg: the
    inner CG preconditioner P_{V,l}), schur_pcg_iters, schur_pcg_tol,
    forward ('kronecker'|'quadrature': the forward problem K x of the Krylov
    loop by the Kronecker-factored kernels or by the quadrature-based
    operator of Sec. 5.3), use_x0 (warm start from the x passed to solve),
    spectrum_gate (Lanczos steps of the set-up check that sigma(P_0^{-1} A~)
    lies in (0, 2); 0 = off), p0_scale (damping factor w of P_0^{-1}),
    breakdown_tol (Krylov breakdown threshold).
    """

    def __init__(self, E, p, nu=1.0, *, c_pen=0.0, schur="Pcq1", schedule="literal",
                 precision="fp64", krylov="minres", restart=50, maxit=1000, order=2,
                 iters=1, max_rhs=1, poll_lag=1, use_graph=False, autotune=True,
                 op_kchunk=0, op_order=-1, fd_plan=-1, op_slabs=0, schur_level=0,
                 schur_pcg_iters=20, schur_pcg_tol=1e-2, op_fused=-1, op_staged=-1,
                 forward="kronecker", use_x0=False, spectrum_gate=0, p0_scale=1.0,
                 breakdown_tol=0.0, op_dma=-1, op_pres_wide=-1, device=None):
        if not torch.cuda.is_available():
            raise RuntimeError("the hyper-power solver runs on a GPU (none visible)")
        self.lib = _lib.load()
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        o = hp_opts()
        self.lib.hp_default_opts(ctypes.byref(o))
        o.c_pen = c_pen
        o.schur_variant = _lib.SCHUR[schur]
        o.l_schedule = _lib.SCHEDULE[schedule]
        o.precision = _lib.PREC[precision]
        o.krylov = _lib.KRYLOV[krylov]
        o.restart = restart
        o.maxit = maxit
        o.order = order
        o.iters = iters
        o.max_rhs = max_rhs
        o.poll_lag = poll_lag
        o.use_graph = int(use_graph)
        o.autotune = int(bool(autotune))
        o.op_kchunk = op_kchunk
        o.op_order = op_order
        o.fd_plan = fd_plan
        o.op_slabs = op_slabs
        o.schur_level = schur_level
        o.schur_pcg_iters = schur_pcg_iters
        o.schur_pcg_tol = schur_pcg_tol
        o.op_fused = op_fused
        o.op_staged = op_staged
        o.forward = {"kronecker": 0, "quadrature": 1}[forward]
        o.use_x0 = int(bool(use_x0))
        o.spectrum_gate = int(spectrum_gate)
        o.p0_scale = float(p0_scale)
        o.breakdown_tol = float(breakdown_tol)
        o.op_dma = int(op_dma)
        o.op_pres_wide = int(op_pres_wide)
        self.opts = o
        self.E, self.p, self.nu = E, p, nu
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.current_stream(self.device)
            ctx = ctypes.c_void_p()
            check(self.lib.hp_setup(E, p, float(nu), ctypes.byref(o),
                                    ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(ctx)),
                  "hp_setup")
        self.ctx = ctx
        dims = (ctypes.c_int64 * 12)()
        offs = (ctypes.c_int64 * 5)()
        check(self.lib.hp_sizes(self.ctx, ctypes.byref(dims), ctypes.byref(offs)), "hp_sizes")
        self.dims = [tuple(dims[3 * b + d] for d in range(3)) for b in range(4)]
        self.offsets = [offs[i] for i in range(5)]
        self.nV = self.offsets[3]
        self.nQ = self.offsets[4] - self.offsets[3]
        self.N = self.offsets[4]
        self.max_rhs = max_rhs

    def tuning(self, nrhs=1):
        """Launch shapes used for batches of `nrhs` (see hp_get_tuning)."""
        t = _lib.hp_tuning()
        check(self.lib.hp_get_tuning(self.ctx, nrhs, ctypes.byref(t)), "hp_get_tuning")
        return {"op_kchunk": t.op_kchunk, "op_order": t.op_order, "op_slabs": t.op_slabs,
                "op_tuned": bool(t.op_tuned),
                "op_us": t.op_us, "fd_plan": list(t.fd_plan), "fd_us": list(t.fd_us),
                "op_staged": t.op_staged, "op_pres_wide": t.op_pres_wide}

    # -- memory helpers ------------------------------------------------------
    def empty(self, n, nrhs=1):
        return torch.empty(nrhs * n, dtype=torch.float64, device=self.device)

    def zeros(self, n, nrhs=1):
        return torch.zeros(nrhs * n, dtype=torch.float64, device=self.device)

    def _nrhs(self, t, n):
        if t.numel() % n:
            raise ValueError(f"size {t.numel()} is not a multiple of {n}")
        return t.numel() // n

    # -- C-ABI calls ----------------------------------------------------------
    def set_nu(self, nu):
        check(self.lib.hp_set_nu(self.ctx, float(nu)), "hp_set_nu")
        self.nu = nu

    def apply_K(self, x, y=None):
        nr = self._nrhs(x, self.N)
        y = self.empty(self.N, nr) if y is None else y
        check(self.lib.hp_apply_K(self.ctx, _ptr(x), _ptr(y), nr), "hp_apply_K")
        return y

    def apply_K_quad(self, x, y=None):
        """y = K x by the quadrature-based (matrix-free) operator, Sec. 5.3."""
        nr = self._nrhs(x, self.N)
        y = self.empty(self.N, nr) if y is None else y
        check(self.lib.hp_apply_K_quad(self.ctx, _ptr(x), _ptr(y), nr), "hp_apply_K_quad")
        return y

    def apply_A(self, u, y=None):
        nr = self._nrhs(u, self.nV)
        y = self.empty(self.nV, nr) if y is None else y
        check(self.lib.hp_apply_A(self.ctx, _ptr(u), _ptr(y), nr), "hp_apply_A")
        return y

    def apply_B(self, p, y=None):
        nr = self._nrhs(p, self.nQ)
        y = self.empty(self.nV, nr) if y is None else y
        check(self.lib.hp_apply_B(self.ctx, _ptr(p), _ptr(y), nr), "hp_apply_B")
        return y

    def apply_Bt(self, u, y=None):
        nr = self._nrhs(u, self.nV)
        y = self.empty(self.nQ, nr) if y is None else y
        check(self.lib.hp_apply_Bt(self.ctx, _ptr(u), _ptr(y), nr), "hp_apply_Bt")
        return y

    def apply_MV(self, u, y=None):
        nr = self._nrhs(u, self.nV)
        y = self.empty(self.nV, nr) if y is None else y
        check(self.lib.hp_apply_MV(self.ctx, _ptr(u), _ptr(y), nr), "hp_apply_MV")
        return y

    def apply_P0(self, x, y=None):
        nr = self._nrhs(x, self.N)
        y = self.empty(self.N, nr) if y is None else y
        check(self.lib.hp_apply_P0(self.ctx, _ptr(x), _ptr(y), nr), "hp_apply_P0")
        return y

    def apply_hyperpower(self, order, iters, x, y=None):
        nr = self._nrhs(x, self.N)
        y = self.empty(self.N, nr) if y is None else y
        check(self.lib.hp_apply_hyperpower(self.ctx, order, iters, _ptr(x), _ptr(y), nr),
              "hp_apply_hyperpower")
        return y

    def apply_PV(self, order, iters, u, y=None):
        """y = P_{V,k}^{-1} u, the velocity block of P_k alone (eq. Pcv)."""
        nr = self._nrhs(u, self.nV)
        y = self.empty(self.nV, nr) if y is None else y
        check(self.lib.hp_apply_PV(self.ctx, order, iters, _ptr(u), _ptr(y), nr), "hp_apply_PV")
        return y

    def spectrum(self, block="velocity", order=2, iters=0, s_level=0, steps=60, start=None,
                 seed=0):
        """Lanczos estimate of the extreme eigenvalues of P_{V,k}^{-1} A
        (block 'velocity') or of P_{Q,k}^{-1} B' P_{V,l}^{-1} B (block
        'schur', l = s_level, constant pressure excluded), k = iters updates
        of order q = order (see hp_spectrum).  start: device vector of the
        block's size (default: seeded standard normal).  Returns a dict with
        lmin, lmax, steps, alpha, beta."""
        from . import synth
        blk = {"velocity": _lib.SPEC_VELOCITY, "schur": _lib.SPEC_SCHUR}[block]
        n = self.nV if blk == _lib.SPEC_VELOCITY else self.nQ
        steps = min(steps, n)
        if start is None:
            start = torch.from_numpy(synth.random_vector(n, seed=seed)).to(self.device)
        if start.numel() != n or start.dtype != torch.float64 or not start.is_contiguous():
            raise ValueError(f"start must be a contiguous float64 vector of {n} entries")
        al = (ctypes.c_double * steps)()
        be = (ctypes.c_double * steps)()
        done = ctypes.c_int()
        lo, hi = ctypes.c_double(), ctypes.c_double()
        check(self.lib.hp_spectrum(self.ctx, blk, order, iters, s_level, steps, _ptr(start),
                                   al, be, ctypes.byref(done), ctypes.byref(lo),
                                   ctypes.byref(hi)), "hp_spectrum")
        m = done.value
        return {"lmin": lo.value, "lmax": hi.value, "steps": m,
                "alpha": np.array(al[:m]), "beta": np.array(be[:m])}

    def solve(self, b, tol=1e-8, x=None, raise_on_noconv=True):
        """hp_solve; with use_x0 the solve starts from (and overwrites) x."""
        nr = self._nrhs(b, self.N)
        if x is None:
            if self.opts.use_x0:
                raise ValueError("use_x0 needs the start vector x")
            x = self.empty(self.N, nr)
        info = hp_solve_info()
        code = self.lib.hp_solve(self.ctx, _ptr(b), _ptr(x), nr, float(tol), ctypes.byref(info))
        if code != 0 and (raise_on_noconv or code != -6):
            check(code, "hp_solve")
        return x, info

    def build_rhs(self, lid, modes=None, b=None, beta=None):
        """Cavity right-hand sides: lid speeds (one per rhs), optional
        body-force modes (amp[nrhs, 3, m], waves[nrhs, 3, m, 3]) and an
        optional body-force coefficient field beta in V_h (n_V per rhs; adds
        M_V beta)."""
        lid = np.ascontiguousarray(np.atleast_1d(np.asarray(lid, dtype=np.float64)))
        nr = lid.size
        b = self.empty(self.N, nr) if b is None else b
        bp = None
        if beta is not None:
            if beta.numel() != nr * self.nV:
                raise ValueError(f"beta must hold {nr} x n_V entries")
            bp = _ptr(beta)
        if modes is None:
            nm, ap, wp = 0, None, None
        else:
            amp, wav = modes
            amp = np.ascontiguousarray(amp, dtype=np.float64)
            wav = np.ascontiguousarray(wav, dtype=np.int32)
            nm = amp.shape[-1]
            ap = amp.ctypes.data_as(ctypes.c_void_p)
            wp = wav.ctypes.data_as(ctypes.c_void_p)
        check(self.lib.hp_build_rhs(self.ctx, lid.ctypes.data_as(ctypes.c_void_p), nm, ap, wp,
                                    bp, _ptr(b), nr), "hp_build_rhs")
        return b

    def grad(self, x, lam, lid):
        nr = self._nrhs(x, self.N)
        lid = np.ascontiguousarray(np.atleast_1d(np.asarray(lid, dtype=np.float64)))
        gb = self.empty(self.nV, nr)
        gn = np.zeros(nr)
        check(self.lib.hp_grad(self.ctx, _ptr(x), _ptr(lam), lid.ctypes.data_as(ctypes.c_void_p),
                               _ptr(gb), gn.ctypes.data_as(ctypes.c_void_p), nr), "hp_grad")
        return gb, gn

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.hp_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
