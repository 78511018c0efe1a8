"""ctypes binding of librexi.so: argument marshalling only.

Every step of the path runs in the library's HIP kernels.  If the library
is not built, or not loadable, every call raises; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, byref, c_double, c_int, c_longlong, c_void_p

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


class RexiError(RuntimeError):
    pass


class RexiParams(ctypes.Structure):
    """Mirror of ``rexi_params`` in include/rexi.h."""
    _fields_ = [("T", c_int), ("nlat", c_int), ("nlon", c_int),
                ("radius", c_double), ("omega", c_double), ("gravity", c_double), ("mean_depth", c_double),
                ("dt", c_double), ("M", c_int), ("h", c_double), ("L", c_int), ("normalize", c_int),
                ("max_states", c_int), ("max_fields", c_int), ("fsphere", c_int), ("f0", c_double)]


def library_path() -> str:
    return os.path.join(_HERE, "librexi.so")


def load_library():
    global _LIB
    if _LIB is not None:
        return _LIB
    path = library_path()
    if not os.path.exists(path):
        raise RexiError(f"{path} is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(path)
    P = c_void_p
    sigs = {
        "rexi_coeffs": [c_int, c_double, c_int, c_int, c_int, P, P, P, POINTER(c_int)],
        "rexi_plan_create": [POINTER(RexiParams), POINTER(c_void_p)],
        "rexi_plan_destroy": [P],
        "rexi_plan_info": [P, POINTER(c_int), POINTER(c_int), POINTER(c_longlong)],
        "rexi_plan_coeffs": [P, P, P, P],
        "sh_forward": [P, P, P, c_int, P],
        "sh_inverse": [P, P, P, c_int, P],
        "sh_vortdiv_to_uv": [P, P, c_longlong, P, c_int, P],
        "sh_uv_to_vortdiv": [P, P, P, c_longlong, c_int, P],
        "rexi_step": [P, P, P, c_int, c_int, P],
        "rexi_step_adjoint": [P, P, P, c_int, c_int, P],
        "rexi_step_per_term": [P, P, P, c_int, P],
        "rexi_step_noalloc": [P, P, P, c_int, c_int, P],
        "rexi_plan_autotune": [P, c_int, P, POINTER(c_int)],
        "rexi_plan_set_schedule": [P, c_int, c_int, POINTER(c_int)],
        "rexi_plan_set_timing": [P, c_int],
        "rexi_plan_set_graphs": [P, c_int],
        "rexi_plan_set_streams": [P, c_int],
        "rexi_plan_kernel_time": [P, c_int, POINTER(c_double), POINTER(c_longlong)],
        "rexi_plan_get_schedule": [P, c_int, POINTER(c_int)],
        "rexi_solve_variants": [c_int, c_int, P, P, P, POINTER(c_int)],
        "rexi_plan_schedule_classes": [P, c_int, c_int, c_int, P, P, P, POINTER(c_int)],
        "rexi_plan_schedule_name": [P, c_int, c_int, ctypes.c_char_p, c_int],
    }
    for name, args in sigs.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = c_int
    lib.rexi_last_error.argtypes = []
    lib.rexi_last_error.restype = ctypes.c_char_p
    _LIB = lib
    return lib


def _check(rc: int, what: str):
    if rc != 0:
        msg = load_library().rexi_last_error().decode()
        raise RexiError(f"{what} failed ({rc}): {msg}")


def rexi_coeffs(M: int, h: float, L: int = 11, normalize: bool = True):
    """Host call: (alpha, beta_plus, beta_minus) complex128 arrays, k = -(M+L)..(M+L)."""
    lib = load_library()
    n = c_int(0)
    _check(lib.rexi_coeffs(M, h, L, int(normalize), 0, None, None, None, byref(n)), "rexi_coeffs")
    out = [np.zeros(n.value, dtype=np.complex128) for _ in range(3)]
    _check(lib.rexi_coeffs(M, h, L, int(normalize), n.value, *(o.ctypes.data for o in out), byref(n)),
           "rexi_coeffs")
    return tuple(out)


def _int_triples(call, what):
    """Run a (capacity, se, kind, st, count) query twice: size, then fill."""
    n = c_int(0)
    _check(call(0, None, None, None, byref(n)), what)
    arrs = [np.zeros(max(1, n.value), dtype=np.int32) for _ in range(3)]
    _check(call(n.value, *(a.ctypes.data for a in arrs), byref(n)), what)
    return [tuple(int(a[i]) for a in arrs) for i in range(n.value)]


def solve_variants(per_term: bool = False):
    """Compiled solve variants as (elements per lane, move kind, states per item)."""
    lib = load_library()
    return _int_triples(lambda cap, a, b, c, n: lib.rexi_solve_variants(int(per_term), cap, a, b, c, n),
                        "rexi_solve_variants")


def params_for(w, max_states=None, max_fields=None, normalize=True, dt=None, grid=True, fsphere=None) -> RexiParams:
    """rexi_params for a workload description (anything with T, nlat, nlon, dt, M, h, L, states).
    ``fsphere``: None for the rotating sphere, else the constant Coriolis parameter f0 (1/s)."""
    import synth
    return RexiParams(T=w.T, nlat=w.nlat if grid else 0, nlon=w.nlon if grid else 0,
                      radius=synth.EARTH_RADIUS, omega=synth.EARTH_OMEGA, gravity=synth.GRAVITY,
                      mean_depth=synth.MEAN_DEPTH, dt=float(w.dt if dt is None else dt), M=w.M, h=w.h, L=w.L,
                      normalize=int(normalize), max_states=max_states or max(1, w.states),
                      max_fields=max_fields or 3 * max(1, w.states),
                      fsphere=0 if fsphere is None else 1, f0=0.0 if fsphere is None else float(fsphere))


def _stream_handle(stream=None):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return c_void_p(s.cuda_stream)


def _need(t, dtype, shape, name):
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be on a GPU")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


class Plan:
    """A rexi_plan: coefficients, operator tables, schedules and workspace."""

    def __init__(self, params: RexiParams):
        lib = load_library()
        self._lib = lib
        self.params = params
        h = c_void_p()
        _check(lib.rexi_plan_create(byref(params), byref(h)), "rexi_plan_create")
        self._h = h
        n, ns, blocks = c_int(), c_int(), c_longlong()
        _check(lib.rexi_plan_info(h, byref(n), byref(ns), byref(blocks)), "rexi_plan_info")
        self.n_poles, self.nspec, self.blocks_per_step = n.value, ns.value, blocks.value

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            _check(self._lib.rexi_plan_destroy(self._h), "rexi_plan_destroy")
            self._h = c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def coeffs(self):
        out = [np.zeros(self.n_poles, dtype=np.complex128) for _ in range(3)]
        _check(self._lib.rexi_plan_coeffs(self._h, *(o.ctypes.data for o in out)), "rexi_plan_coeffs")
        return tuple(out)

    def _state_call(self, fn, name, u0, nsteps, out, stream):
        import torch
        S = u0.shape[0] if u0.dim() == 3 else -1
        _need(u0, torch.complex128, (S, 3, self.nspec), "input state")
        if out is None:
            out = torch.empty_like(u0)
        _need(out, torch.complex128, (S, 3, self.nspec), "output state")
        args = [self._h, c_void_p(u0.data_ptr()), c_void_p(out.data_ptr()), S]
        if nsteps is not None:
            args.append(int(nsteps))
        args.append(_stream_handle(stream))
        _check(fn(*args), name)
        return out

    def step(self, u0, nsteps: int = 1, out=None, stream=None):
        """u1 = R^nsteps u0 (rexi_step)."""
        return self._state_call(self._lib.rexi_step, "rexi_step", u0, nsteps, out, stream)

    def step_adjoint(self, g1, nsteps: int = 1, out=None, stream=None):
        """g0 = (R^H)^nsteps g1 (rexi_step_adjoint)."""
        return self._state_call(self._lib.rexi_step_adjoint, "rexi_step_adjoint", g1, nsteps, out, stream)

    def step_noalloc(self, u0, nsteps: int = 1, out=None, stream=None):
        """u1 = R^nsteps u0 with the library's fixed workspace (rexi_step_noalloc).
        ``out`` must be given by callers that cannot allocate."""
        return self._state_call(self._lib.rexi_step_noalloc, "rexi_step_noalloc", u0, nsteps, out, stream)

    def step_per_term(self, u0, out=None, stream=None):
        """One step in the plain per-term launch form (rexi_step_per_term)."""
        return self._state_call(self._lib.rexi_step_per_term, "rexi_step_per_term", u0, None, out, stream)

    def sh_forward(self, grid, out=None, stream=None):
        import torch
        B = grid.shape[0] if grid.dim() == 3 else -1
        _need(grid, torch.float64, (B, self.params.nlat, self.params.nlon), "grid")
        if out is None:
            out = torch.empty((B, self.nspec), dtype=torch.complex128, device=grid.device)
        _need(out, torch.complex128, (B, self.nspec), "spec")
        _check(self._lib.sh_forward(self._h, c_void_p(grid.data_ptr()), c_void_p(out.data_ptr()), B,
                                    _stream_handle(stream)), "sh_forward")
        return out

    def sh_inverse(self, spec, out=None, stream=None):
        import torch
        B = spec.shape[0] if spec.dim() == 2 else -1
        _need(spec, torch.complex128, (B, self.nspec), "spec")
        if out is None:
            out = torch.empty((B, self.params.nlat, self.params.nlon), dtype=torch.float64, device=spec.device)
        _need(out, torch.float64, (B, self.params.nlat, self.params.nlon), "grid")
        _check(self._lib.sh_inverse(self._h, c_void_p(spec.data_ptr()), c_void_p(out.data_ptr()), B,
                                    _stream_handle(stream)), "sh_inverse")
        return out

    def _vd_view(self, vd, name):
        """(pointer to zeta of pair 0, stride in complex entries, B) of a
        [B][2][nspec] (zeta, delta) tensor or a [S][3][nspec] state tensor."""
        import torch
        if vd.dim() != 3 or vd.shape[1] not in (2, 3):
            raise ValueError(f"{name} must have shape (B, 2, nspec) or (S, 3, nspec), got {tuple(vd.shape)}")
        B, k = vd.shape[0], vd.shape[1]
        _need(vd, torch.complex128, (B, k, self.nspec), name)
        off = (k - 2) * self.nspec * 16
        return c_void_p(vd.data_ptr() + off), k * self.nspec, B

    def vortdiv_to_uv(self, vd, out=None, stream=None):
        """Winds (u, v) [B][2][nlat][nlon] from vorticity and divergence
        (sh_vortdiv_to_uv).  vd: [B][2][nspec] (zeta, delta) or states
        [S][3][nspec] (Phi, zeta, delta)."""
        import torch
        ptr, stride, B = self._vd_view(vd, "vd")
        shape = (B, 2, self.params.nlat, self.params.nlon)
        if out is None:
            out = torch.empty(shape, dtype=torch.float64, device=vd.device)
        _need(out, torch.float64, shape, "uv")
        _check(self._lib.sh_vortdiv_to_uv(self._h, ptr, stride, c_void_p(out.data_ptr()), B,
                                          _stream_handle(stream)), "sh_vortdiv_to_uv")
        return out

    def uv_to_vortdiv(self, uv, out=None, stream=None):
        """Vorticity and divergence of winds uv [B][2][nlat][nlon]
        (sh_uv_to_vortdiv).  out: [B][2][nspec], or states [B][3][nspec] whose
        zeta and delta rows are written (Phi untouched)."""
        import torch
        B = uv.shape[0] if uv.dim() == 4 else -1
        _need(uv, torch.float64, (B, 2, self.params.nlat, self.params.nlon), "uv")
        if out is None:
            out = torch.empty((B, 2, self.nspec), dtype=torch.complex128, device=uv.device)
        ptr, stride, Bo = self._vd_view(out, "vd")
        if Bo != B:
            raise ValueError(f"vd holds {Bo} pairs, uv {B}")
        _check(self._lib.sh_uv_to_vortdiv(self._h, c_void_p(uv.data_ptr()), ptr, stride, B,
                                          _stream_handle(stream)), "sh_uv_to_vortdiv")
        return out

    def autotune(self, S: int, stream=None) -> int:
        c = c_int(-1)
        _check(self._lib.rexi_plan_autotune(self._h, S, _stream_handle(stream), byref(c)), "rexi_plan_autotune")
        return c.value

    def schedule_count(self, S: int) -> int:
        n = c_int(0)
        _check(self._lib.rexi_plan_set_schedule(self._h, S, -1, byref(n)), "rexi_plan_set_schedule")
        return n.value

    def chosen_schedule(self, S: int) -> int:
        """Index of the schedule candidate that steps with S states use now."""
        i = c_int(-1)
        _check(self._lib.rexi_plan_get_schedule(self._h, S, byref(i)), "rexi_plan_get_schedule")
        return i.value

    def schedule_classes(self, S: int, index: int):
        """(elements per lane, move kind, states per item) of each solve launch
        of schedule ``index`` (-1: the per-term schedule)."""
        return _int_triples(lambda cap, a, b, c, n: self._lib.rexi_plan_schedule_classes(
            self._h, S, index, cap, a, b, c, n), "rexi_plan_schedule_classes")

    def schedule_name(self, S: int, index: int) -> str:
        """Name of schedule ``index`` (-1: the per-term schedule): tile policy,
        item count, persistent or not, states sharing factorisations."""
        buf = ctypes.create_string_buffer(128)
        _check(self._lib.rexi_plan_schedule_name(self._h, S, index, buf, len(buf)), "rexi_plan_schedule_name")
        return buf.value.decode()

    def set_schedule(self, S: int, index: int):
        _check(self._lib.rexi_plan_set_schedule(self._h, S, index, None), "rexi_plan_set_schedule")

    KERNEL_SOLVE, KERNEL_LEGENDRE_FWD, KERNEL_LEGENDRE_INV = 0, 1, 2

    def set_graphs(self, enable: bool):
        _check(self._lib.rexi_plan_set_graphs(self._h, int(enable)), "rexi_plan_set_graphs")

    def set_streams(self, enable: bool):
        """Tile-class launches concurrent on side streams (True, default) or serial."""
        _check(self._lib.rexi_plan_set_streams(self._h, int(enable)), "rexi_plan_set_streams")

    def set_timing(self, enable: bool):
        _check(self._lib.rexi_plan_set_timing(self._h, int(enable)), "rexi_plan_set_timing")

    def kernel_time(self, kernel: int):
        """(total ms, launches) of one timed kernel since the last query."""
        ms, n = c_double(0), c_longlong(0)
        _check(self._lib.rexi_plan_kernel_time(self._h, kernel, byref(ms), byref(n)), "rexi_plan_kernel_time")
        return ms.value, n.value


def plan_for(w, **kw) -> Plan:
    return Plan(params_for(w, **kw))


def _step_function():
    import torch

    class _Step(torch.autograd.Function):
        """u1 = R^nsteps u0 with a hand-written adjoint: grad_u0 = (R^H)^nsteps grad_u1."""

        @staticmethod
        def forward(ctx, u0, plan, nsteps):
            ctx.plan = plan
            ctx.nsteps = nsteps
            return plan.step(u0.contiguous(), nsteps)

        @staticmethod
        def backward(ctx, g1):
            return ctx.plan.step_adjoint(g1.contiguous(), ctx.nsteps), None, None

    return _Step


_STEP = None


def Step():
    """The torch.autograd.Function class (created on first use)."""
    global _STEP
    if _STEP is None:
        _STEP = _step_function()
    return _STEP


def run(plan: Plan, u0, nsteps: int, checkpoint_every: int = 0):
    """Differentiable nsteps-step integration.

    The steps are applied in segments of ``checkpoint_every`` steps (all at
    once if 0); autograd keeps only the segment-boundary states, and since
    the map is linear its backward pass needs none of them: each segment's
    backward is one adjoint call."""
    k = nsteps if checkpoint_every <= 0 else checkpoint_every
    u = u0
    done = 0
    S = Step()
    while done < nsteps:
        n = min(k, nsteps - done)
        u = S.apply(u, plan, n)
        done += n
    return u
