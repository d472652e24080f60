"""Python binding of libpwdf (the C ABI in include/pwdf.h).

Argument marshalling only: every step of the long-range J build runs in the HIP
kernels of libpwdf.so.  PyTorch supplies device memory and the current HIP
stream.  If the library is missing this module raises at import of the
library; there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "libpwdf.so")

PWDF_FP64 = 0
PWDF_FP32_MFMA = 1

_STATUS = {0: "PWDF_OK", -1: "PWDF_EINVAL", -2: "PWDF_ENOMEM", -3: "PWDF_EDEVICE",
           -4: "PWDF_EUNSUPPORTED", -5: "PWDF_ENONFINITE", -6: "PWDF_ESTATE"}

PWDF_JK_FULL = 0
PWDF_JK_SUPPORT = 1
PWDF_JK_PACKED = 2

PWDF_DK_FULL = 0
PWDF_DK_PACKED = 1

EXPORTED = ["pwdf_create", "pwdf_query", "pwdf_build_j", "pwdf_build_j_graph", "pwdf_get_rhoG", "pwdf_grad",
            "pwdf_autotune", "pwdf_last_error", "pwdf_destroy", "pwdf_plan_stats",
            "pwdf_profile_enable", "pwdf_profile_read", "pwdf_set_jk_layout", "pwdf_check_input",
            "pwdf_get_jk_support", "pwdf_build_j_noalloc", "pwdf_set_fp32_head", "pwdf_energy_real",
            "pwdf_debug_fail_alloc", "pwdf_debug_live_allocs", "pwdf_set_dk_layout"]


class PwdfError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class Screen(ctypes.Structure):
    _fields_ = [("eps_pair", ctypes.c_double), ("eps_G", ctypes.c_double), ("r_max", ctypes.c_double),
                ("pair_gcut", ctypes.c_int), ("alpha_cut", ctypes.c_double), ("dd_gpw", ctypes.c_int)]


def _screen(prob) -> Screen:
    return Screen(prob.eps_pair, prob.eps_G, prob.r_max, int(getattr(prob, "pair_gcut", 0)),
                  float(getattr(prob, "alpha_cut", 0.0)), int(getattr(prob, "dd_gpw", 0)))


class Stats(ctypes.Structure):
    _fields_ = [("npairs_by_class", ctypes.c_int64 * 16), ("nG", ctypes.c_int64), ("npairs", ctypes.c_int64),
                ("nbf", ctypes.c_int64), ("nk", ctypes.c_int64), ("nimg", ctypes.c_int64),
                ("nblocks", ctypes.c_int64), ("nseg", ctypes.c_int64), ("pairG_evals", ctypes.c_double),
                ("t_us", ctypes.c_double * 8), ("seg_len", ctypes.c_int64),
                ("fork", ctypes.c_int64), ("jk_support", ctypes.c_int64), ("dk_support", ctypes.c_int64),
                ("jk_layout", ctypes.c_int64), ("nG_head", ctypes.c_int64), ("pairG_head", ctypes.c_double),
                ("npairs_dd", ctypes.c_int64), ("gpw_grid", ctypes.c_int64 * 3)]

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_ if f not in ("npairs_by_class", "t_us", "gpw_grid")}
        d["gpw_grid"] = tuple(int(x) for x in self.gpw_grid)
        d["npairs_by_class"] = {f"{c // 4}{c % 4}": int(self.npairs_by_class[c]) for c in range(16)
                                if self.npairs_by_class[c]}
        return d


class KProf(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_int64), ("ms", ctypes.c_double),
                ("units", ctypes.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIBPATH):
            raise ImportError(f"libpwdf.so is not built ({LIBPATH}); run __graft_entry__.build()")
        L = ctypes.CDLL(LIBPATH)
        vp, dp, ip = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)
        L.pwdf_create.restype = ctypes.c_int
        L.pwdf_create.argtypes = [ctypes.POINTER(vp), dp, ctypes.c_int, dp, ctypes.c_int, ip, ip, ip, dp, dp, ip,
                                  ctypes.c_double, ctypes.POINTER(Screen), ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.pwdf_plan_stats.restype = ctypes.c_int
        L.pwdf_plan_stats.argtypes = [dp, ctypes.c_int, dp, ctypes.c_int, ip, ip, ip, dp, dp, ip,
                                      ctypes.c_double, ctypes.POINTER(Screen), ctypes.POINTER(Stats)]
        L.pwdf_query.restype = ctypes.c_int
        L.pwdf_query.argtypes = [vp, ctypes.POINTER(Stats)]
        L.pwdf_build_j.restype = ctypes.c_int
        L.pwdf_build_j.argtypes = [vp, ctypes.c_int, vp, vp, vp, vp]
        L.pwdf_build_j_noalloc.restype = ctypes.c_int
        L.pwdf_build_j_noalloc.argtypes = [vp, ctypes.c_int, vp, vp, vp, vp]
        L.pwdf_build_j_graph.restype = ctypes.c_int
        L.pwdf_build_j_graph.argtypes = [vp, ctypes.c_int, vp, vp, vp, vp]
        L.pwdf_get_rhoG.restype = ctypes.c_int
        L.pwdf_get_rhoG.argtypes = [vp, ctypes.c_int, vp, vp, ip, vp]
        L.pwdf_grad.restype = ctypes.c_int
        L.pwdf_grad.argtypes = [vp, ctypes.c_int, vp, vp, vp, vp]
        L.pwdf_autotune.restype = ctypes.c_int
        L.pwdf_autotune.argtypes = [vp, ctypes.c_int, ctypes.c_char_p]
        L.pwdf_profile_enable.restype = ctypes.c_int
        L.pwdf_profile_enable.argtypes = [vp, ctypes.c_int]
        L.pwdf_profile_read.restype = ctypes.c_int
        L.pwdf_profile_read.argtypes = [vp, ctypes.POINTER(KProf), ctypes.c_int, ip]
        L.pwdf_set_jk_layout.restype = ctypes.c_int
        L.pwdf_set_jk_layout.argtypes = [vp, ctypes.c_int]
        L.pwdf_set_dk_layout.restype = ctypes.c_int
        L.pwdf_set_dk_layout.argtypes = [vp, ctypes.c_int]
        L.pwdf_set_fp32_head.restype = ctypes.c_int
        L.pwdf_set_fp32_head.argtypes = [vp, ctypes.c_double]
        L.pwdf_energy_real.restype = ctypes.c_int
        L.pwdf_energy_real.argtypes = [vp, ctypes.c_int, vp, vp]
        L.pwdf_debug_fail_alloc.restype = None
        L.pwdf_debug_fail_alloc.argtypes = [ctypes.c_int]
        L.pwdf_debug_live_allocs.restype = ctypes.c_int64
        L.pwdf_debug_live_allocs.argtypes = []
        L.pwdf_get_jk_support.restype = ctypes.c_int
        L.pwdf_get_jk_support.argtypes = [vp, ip, ip]
        L.pwdf_check_input.restype = ctypes.c_int
        L.pwdf_check_input.argtypes = [vp, vp]
        L.pwdf_last_error.restype = ctypes.c_char_p
        L.pwdf_last_error.argtypes = [vp]
        L.pwdf_destroy.restype = None
        L.pwdf_destroy.argtypes = [vp]
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def _basis_arrays(prob):
    return dict(
        lat=np.ascontiguousarray(prob.lattice, dtype=np.float64).ravel(),
        xyz=np.ascontiguousarray(prob.xyz, dtype=np.float64).ravel(),
        sa=np.ascontiguousarray(prob.shell_atom, dtype=np.int32),
        sl=np.ascontiguousarray(prob.shell_l, dtype=np.int32),
        sn=np.ascontiguousarray(prob.shell_nprim, dtype=np.int32),
        ex=np.ascontiguousarray(prob.exps, dtype=np.float64),
        co=np.ascontiguousarray(prob.coefs, dtype=np.float64),
        km=np.ascontiguousarray(prob.kmesh, dtype=np.int32),
    )


def plan_stats(prob) -> dict:
    """Host-only plan sizes (no device needed)."""
    a = _basis_arrays(prob)
    st = Stats()
    scr = _screen(prob)
    rc = lib().pwdf_plan_stats(_dp(a["lat"]), prob.natm, _dp(a["xyz"]), prob.nshell, _ip(a["sa"]), _ip(a["sl"]),
                               _ip(a["sn"]), _dp(a["ex"]), _dp(a["co"]), _ip(a["km"]), float(prob.omega),
                               ctypes.byref(scr), ctypes.byref(st))
    if rc != 0:
        raise PwdfError(rc, lib().pwdf_last_error(None).decode())
    return st.as_dict()


class LongRangeJ:
    """One plan (geometry, basis, k-mesh, omega) on one device."""

    def __init__(self, prob, precision: int = PWDF_FP64, max_ndm: int = 1, device: int = 0):
        self.prob = prob
        self.precision = precision
        self.max_ndm = max_ndm
        self.device = device
        self._last_ndm = 0
        a = _basis_arrays(prob)
        self._keep = a
        scr = _screen(prob)
        h = ctypes.c_void_p()
        rc = lib().pwdf_create(ctypes.byref(h), _dp(a["lat"]), prob.natm, _dp(a["xyz"]), prob.nshell, _ip(a["sa"]),
                               _ip(a["sl"]), _ip(a["sn"]), _dp(a["ex"]), _dp(a["co"]), _ip(a["km"]),
                               float(prob.omega), ctypes.byref(scr), int(precision), int(max_ndm), int(device))
        if rc != 0:
            raise PwdfError(rc, lib().pwdf_last_error(None).decode())
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().pwdf_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _err(self, rc):
        raise PwdfError(rc, lib().pwdf_last_error(self._h).decode())

    def stats(self) -> dict:
        st = Stats()
        rc = lib().pwdf_query(self._h, ctypes.byref(st))
        if rc != 0:
            self._err(rc)
        return st.as_dict()

    @staticmethod
    def _stream(stream):
        import torch
        s = torch.cuda.current_stream() if stream is None else stream
        return ctypes.c_void_p(s.cuda_stream)

    def _check_D(self, Dk):
        import torch
        p = self.prob
        if Dk.dtype != torch.complex128 or not Dk.is_cuda or not Dk.is_contiguous():
            raise ValueError("Dk must be a contiguous complex128 CUDA tensor")
        if getattr(self, "_dk_layout", PWDF_DK_FULL) == PWDF_DK_PACKED:
            if Dk.dim() == 2:
                Dk = Dk.unsqueeze(0)
            ns = self.stats()["jk_support"]
            if tuple(Dk.shape[1:]) != (p.nk, ns):
                raise ValueError(f"packed Dk shape {tuple(Dk.shape)} != [ndm, {p.nk}, {ns}]")
            return Dk
        if Dk.dim() == 3:
            Dk = Dk.unsqueeze(0)
        if tuple(Dk.shape[1:]) != (p.nk, p.nbf, p.nbf):
            raise ValueError(f"Dk shape {tuple(Dk.shape)} != [ndm, {p.nk}, {p.nbf}, {p.nbf}]")
        return Dk

    def set_fp32_head(self, weight: float):
        """FP32-MFMA form: G vectors with v(G) >= weight * max v take FP64 tiles
        (default 2^-20); rebuilds the workspaces."""
        rc = lib().pwdf_set_fp32_head(self._h, float(weight))
        if rc != 0:
            self._err(rc)

    def set_jk_layout(self, layout: int):
        """PWDF_JK_FULL (every element of J(k) written), PWDF_JK_SUPPORT (only the
        pair support; a J(k) buffer passed in must have been cleared once) or
        PWDF_JK_PACKED (J(k) as [ndm][nk][jk_support], element order of
        jk_support())."""
        rc = lib().pwdf_set_jk_layout(self._h, int(layout))
        if rc != 0:
            self._err(rc)
        self._jk_layout = int(layout)

    def set_dk_layout(self, layout: int):
        """PWDF_DK_FULL (D(k) as [ndm][nk][nbf][nbf]) or PWDF_DK_PACKED (D(k) as
        [ndm][nk][jk_support], the element order of jk_support(); pack_dk makes it)."""
        rc = lib().pwdf_set_dk_layout(self._h, int(layout))
        if rc != 0:
            self._err(rc)
        self._dk_layout = int(layout)

    def pack_dk(self, Dk):
        """[ndm][nk][jk_support] values of a dense [ndm][nk][nbf][nbf] D(k) (a gather
        on the device, outside the library)."""
        import torch
        mu, nu = self.jk_support()
        p = self.prob
        idx = torch.from_numpy(mu.astype(np.int64) * p.nbf + nu).to(Dk.device)
        D = Dk if Dk.dim() == 4 else Dk.unsqueeze(0)
        return D.reshape(D.shape[0], p.nk, p.nbf * p.nbf).index_select(2, idx).contiguous()

    def jk_support(self):
        """(mu, nu) int arrays of the packed J(k) element order."""
        n = self.stats()["jk_support"]
        mu = np.zeros(max(n, 1), dtype=np.int32)
        nu = np.zeros(max(n, 1), dtype=np.int32)
        rc = lib().pwdf_get_jk_support(self._h, _ip(mu), _ip(nu))
        if rc != 0:
            self._err(rc)
        return mu[:n], nu[:n]

    def unpack_jk(self, Jp):
        """Dense [ndm][nk][nbf][nbf] J(k) (zeros off the support) from the packed layout."""
        import torch
        mu, nu = self.jk_support()
        p = self.prob
        idx = torch.from_numpy(mu.astype(np.int64) * p.nbf + nu).to(Jp.device)
        out = torch.zeros((Jp.shape[0], p.nk, p.nbf * p.nbf), dtype=Jp.dtype, device=Jp.device)
        out[:, :, idx] = Jp
        return out.view(Jp.shape[0], p.nk, p.nbf, p.nbf)

    def check_input(self, stream=None):
        """Raises PwdfError(PWDF_ENONFINITE) if a call since the last check read a
        non-finite D(k) value on the pair support (synchronises the stream)."""
        rc = lib().pwdf_check_input(self._h, self._stream(stream))
        if rc != 0:
            self._err(rc)

    def build_j(self, Dk, Jk=None, EJ=None, stream=None, graph=False, noalloc=False):
        """Dk: complex128 [ndm][nk][nbf][nbf] (or [nk][nbf][nbf]) on the device.
        Returns (Jk, EJ) device tensors; enqueued on `stream` (default: current).
        graph=True goes through pwdf_build_j_graph (captured once per set of
        buffers, then replayed): pass the same Jk / EJ tensors on every call.
        In the support layout a J(k) allocated here starts as zeros.
        noalloc=True goes through pwdf_build_j_noalloc (workspaces in the
        library's static device scratch; pass Jk and EJ to allocate nothing)."""
        import torch
        Dk = self._check_D(Dk)
        ndm = Dk.shape[0]
        if Jk is None:
            layout = getattr(self, "_jk_layout", PWDF_JK_FULL)
            if layout == PWDF_JK_PACKED:
                Jk = torch.empty((ndm, self.prob.nk, self.stats()["jk_support"]), dtype=Dk.dtype, device=Dk.device)
            elif layout == PWDF_JK_SUPPORT:
                Jk = torch.zeros((ndm, self.prob.nk, self.prob.nbf, self.prob.nbf), dtype=Dk.dtype,
                                 device=Dk.device)
            else:
                Jk = torch.empty((ndm, self.prob.nk, self.prob.nbf, self.prob.nbf), dtype=Dk.dtype,
                                 device=Dk.device)
        if EJ is None:
            EJ = torch.empty(ndm, dtype=torch.float64, device=Dk.device)
        fn = lib().pwdf_build_j_graph if graph else lib().pwdf_build_j
        if noalloc:
            fn = lib().pwdf_build_j_noalloc
        rc = fn(self._h, ndm, ctypes.c_void_p(Dk.data_ptr()), ctypes.c_void_p(Jk.data_ptr()),
                ctypes.c_void_p(EJ.data_ptr()), self._stream(stream))
        if rc != 0:
            self._err(rc)
        self._last_ndm = ndm
        return Jk, EJ

    def energy_real(self, ndm=None, stream=None):
        """E_J^(R) = 1/2 sum D(L) J(L) of the last build_j (eager or graph) on this
        context, [ndm] device tensor; ndm defaults to that build's."""
        import torch
        n = self._last_ndm if ndm is None else ndm
        ER = torch.empty(max(1, n), dtype=torch.float64, device=torch.device("cuda", self.device))
        rc = lib().pwdf_energy_real(self._h, n, ctypes.c_void_p(ER.data_ptr()), self._stream(stream))
        if rc != 0:
            self._err(rc)
        return ER

    def get_rhoG(self, Dk, stream=None):
        """rho(G) on the half space the kernels walk, and the Miller indices (host)."""
        import torch
        Dk = self._check_D(Dk)
        ndm = Dk.shape[0]
        nh = self.stats()["nG"] // 2
        rho = torch.empty((ndm, nh), dtype=torch.complex128, device=Dk.device)
        miller = np.zeros((nh, 3), dtype=np.int32)
        rc = lib().pwdf_get_rhoG(self._h, ndm, ctypes.c_void_p(Dk.data_ptr()), ctypes.c_void_p(rho.data_ptr()),
                                 _ip(miller), self._stream(stream))
        if rc != 0:
            self._err(rc)
        return rho, miller

    def grad(self, Dk, stream=None):
        """dE_J/dR [ndm][natm][3] and E_J [ndm] (device tensors)."""
        import torch
        Dk = self._check_D(Dk)
        ndm = Dk.shape[0]
        g = torch.empty((ndm, self.prob.natm, 3), dtype=torch.float64, device=Dk.device)
        EJ = torch.empty(ndm, dtype=torch.float64, device=Dk.device)
        rc = lib().pwdf_grad(self._h, ndm, ctypes.c_void_p(Dk.data_ptr()), ctypes.c_void_p(g.data_ptr()),
                             ctypes.c_void_p(EJ.data_ptr()), self._stream(stream))
        if rc != 0:
            self._err(rc)
        return g, EJ

    def profile_enable(self, on: bool = True):
        rc = lib().pwdf_profile_enable(self._h, 1 if on else 0)
        if rc != 0:
            self._err(rc)

    def profile_read(self) -> dict:
        """{kernel name: {"launches", "ms", "units"}} accumulated since profile_enable."""
        n = ctypes.c_int(0)
        rc = lib().pwdf_profile_read(self._h, None, 0, ctypes.byref(n))
        if rc != 0:
            self._err(rc)
        arr = (KProf * max(1, n.value))()
        rc = lib().pwdf_profile_read(self._h, arr, n.value, ctypes.byref(n))
        if rc != 0:
            self._err(rc)
        return {arr[i].name.decode(): dict(launches=int(arr[i].launches), ms=float(arr[i].ms),
                                           units=float(arr[i].units)) for i in range(n.value)}

    def autotune(self, ndm: int = 1, cache_path: Optional[str] = None):
        rc = lib().pwdf_autotune(self._h, int(ndm), cache_path.encode() if cache_path else None)
        if rc != 0:
            self._err(rc)


def _autograd_function():
    import torch

    class LongRangeJEnergy(torch.autograd.Function):
        """E_J[ndm] = LongRangeJEnergy.apply(Dk, xyz, plan).

        Dk: complex128 [ndm][nk][nbf][nbf] on the device; xyz: float64 [natm][3]
        (must equal the geometry the plan was built for: the pair list and G set
        stay those of the plan, as in the gradient definition at fixed pair list).
        backward: dE/dD(k) = w_k conj J(k) (torch's convention for complex inputs,
        from the symmetric bilinear form E = 1/2 sum_k w_k sum D(k) J(k)) and
        dE/dR from the adjoint kernels of pwdf_grad.
        """

        @staticmethod
        def forward(ctx, Dk, xyz, plan):
            ref = np.asarray(plan.prob.xyz, dtype=np.float64)
            got = xyz.detach().to("cpu", torch.float64).numpy()
            if got.shape != ref.shape or not np.array_equal(got, ref):
                raise ValueError("xyz differs from the geometry of the plan; build a new LongRangeJ")
            if getattr(plan, "_dk_layout", PWDF_DK_FULL) != PWDF_DK_FULL:
                raise ValueError("long_range_energy takes a dense D(k): set PWDF_DK_FULL")
            Jk, EJ = plan.build_j(Dk)
            if getattr(plan, "_jk_layout", PWDF_JK_FULL) == PWDF_JK_PACKED:
                Jk = plan.unpack_jk(Jk)
            ctx.save_for_backward(Dk, Jk)
            ctx.plan = plan
            ctx.xyz_meta = (xyz.device, xyz.dtype)
            return EJ

        @staticmethod
        def backward(ctx, gE):
            Dk, Jk = ctx.saved_tensors
            plan = ctx.plan
            grad_D = grad_x = None
            gE = gE.to(torch.float64)
            if ctx.needs_input_grad[0]:
                w = 1.0 / plan.prob.nk
                grad_D = (gE.view(-1, 1, 1, 1) * w) * Jk.conj()
                if Dk.dim() == 3:
                    grad_D = grad_D[0]
            if ctx.needs_input_grad[1]:
                g, _ = plan.grad(Dk)
                grad_x = (gE.view(-1, 1, 1) * g).sum(0).to(ctx.xyz_meta[0], ctx.xyz_meta[1])
            return grad_D, grad_x, None

    return LongRangeJEnergy


_LRJE = None


def long_range_energy(Dk, xyz, plan):
    """Differentiable E_J (see LongRangeJEnergy)."""
    global _LRJE
    if _LRJE is None:
        _LRJE = _autograd_function()
    return _LRJE.apply(Dk, xyz, plan)
