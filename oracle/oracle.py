"""ctypes front end of the FP64 CPU oracle (test infrastructure only).

Only tests/, the smoke check and the benchmark's CPU-baseline leg may import
this module.  It loads oracle/liboracle.so, which `build()` compiles from
oracle/pwdf_oracle.c with plain gcc (no GPU code, nothing shared with the HIP
library).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "pwdf_oracle.c")
LIB = os.environ.get("PWDF_ORACLE_LIB", os.path.join(HERE, "liboracle.so"))

_lib = None


def build(force: bool = True) -> str:
    if force or not os.path.exists(LIB):
        cmd = ["gcc", "-O2", "-fopenmp", "-fno-fast-math", "-ffp-contract=off", "-std=c11",
               "-shared", "-fPIC", "-o", LIB + ".tmp", SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(LIB + ".tmp", LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = ctypes.CDLL(LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        L.orc_build_j.restype = ctypes.c_int
        L.orc_build_j.argtypes = [dp, ctypes.c_int, dp, ctypes.c_int, ip, ip, ip, dp, dp, ip,
                                  ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                  dp, dp, dp, dp, ip, ctypes.c_int, ip, dp, ctypes.c_int, ctypes.c_int,
                                  ctypes.c_double]
        L.orc_sizes.restype = ctypes.c_int
        L.orc_sizes.argtypes = [dp, ctypes.c_int, dp, ctypes.c_int, ip, ip, ip, dp, dp, ip,
                                ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                ctypes.POINTER(ctypes.c_int64)]
        L.orc_pairs.restype = ctypes.c_int
        L.orc_pairs.argtypes = [dp, ctypes.c_int, dp, ctypes.c_int, ip, ip, ip, dp, dp, ip,
                                ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                ip, ctypes.c_int]
        L.orc_pair_cut.restype = None
        L.orc_pair_cut.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, dp, ctypes.c_double, dp,
                                   ctypes.c_double, ctypes.c_double, ctypes.c_double, dp]
        L.orc_ft_axis.restype = None
        L.orc_ft_axis.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                  ctypes.c_double, ctypes.c_double, ctypes.c_double, dp]
        L.orc_pair_ft.restype = None
        L.orc_pair_ft.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, dp, ctypes.c_double,
                                  dp, dp, dp, dp, dp]
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _i(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def _prob_args(prob):
    arrs = dict(
        lat=np.ascontiguousarray(prob.lattice, dtype=np.float64).ravel(),
        xyz=np.ascontiguousarray(prob.xyz, dtype=np.float64).ravel(),
        sa=np.ascontiguousarray(prob.shell_atom, dtype=np.int32),
        sl=np.ascontiguousarray(prob.shell_l, dtype=np.int32),
        sn=np.ascontiguousarray(prob.shell_nprim, dtype=np.int32),
        ex=np.ascontiguousarray(prob.exps, dtype=np.float64),
        co=np.ascontiguousarray(prob.coefs, dtype=np.float64),
        km=np.ascontiguousarray(prob.kmesh, dtype=np.int32),
    )
    args = [_d(arrs["lat"]), prob.natm, _d(arrs["xyz"]), prob.nshell, _i(arrs["sa"]), _i(arrs["sl"]),
            _i(arrs["sn"]), _d(arrs["ex"]), _d(arrs["co"]), _i(arrs["km"]), float(prob.omega),
            float(prob.eps_pair), float(prob.eps_G), float(prob.r_max)]
    return arrs, args


def sizes(prob):
    arrs, args = _prob_args(prob)
    out = np.zeros(4, dtype=np.int64)
    rc = lib().orc_sizes(*args, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    if rc != 0:
        raise ValueError(f"oracle rejected the problem ({rc})")
    return dict(nG=int(out[0]), npairs=int(out[1]), nbf=int(out[2]), nk=int(out[3]))


def pairs(prob):
    """The oracle's screened pair list, int [npairs][7]: sa, sb, ia, ib, m1, m2, m3."""
    arrs, args = _prob_args(prob)
    n = lib().orc_pairs(*args, ctypes.POINTER(ctypes.c_int)(), 0)
    if n < 0:
        raise ValueError(f"oracle rejected the problem ({n})")
    out = np.zeros((max(n, 1), 7), dtype=np.int32)
    lib().orc_pairs(*args, _i(out), n)
    return out[:n]


class OracleResult(dict):
    pass


def build_j(prob, Dk, *, want_J=True, want_rho=True, want_grad=False, nthreads=0, pair_gcut=None,
            alpha_cut=None):
    """Long-range J, energies, rho(G) and (optionally) dE/dR for one density.
    pair_gcut (default: prob.pair_gcut): each screened pair sees only the G
    vectors inside its own cut radius (section "Integral screening").
    alpha_cut (default: prob.alpha_cut; <= 0 off): compact/diffuse classification
    (section "Density classification: compact and diffuse"): pairs of two
    primitives with exponents below alpha_cut interact in full (4 pi/G^2), the
    others keep the long-range kernel among themselves; rho is then rho_C + rho_D.

    Dk: complex128 [nk][nbf][nbf].  Returns dict with J (complex [nk][nbf][nbf]),
    E_real, E_G, E_k, maxImJ, maxJ, charge (Omega rho(0)), rho (complex [nG]),
    miller (int [nG][3]), grad ([natm][3]).
    """
    arrs, args = _prob_args(prob)
    Dk = np.ascontiguousarray(Dk, dtype=np.complex128)
    nk, nbf = prob.nk, prob.nbf
    assert Dk.shape == (nk, nbf, nbf), Dk.shape
    Dv = Dk.view(np.float64)
    J = np.zeros((nk, nbf, nbf), dtype=np.complex128) if want_J else None
    energy = np.zeros(6)
    nG = sizes(prob)["nG"] if want_rho else 0
    rho = np.zeros((max(nG, 1), 2)) if want_rho else None
    miller = np.zeros((max(nG, 1), 3), dtype=np.int32) if want_rho else None
    nG_out = ctypes.c_int(0)
    grad = np.zeros((prob.natm, 3)) if want_grad else None
    null_d = ctypes.POINTER(ctypes.c_double)()
    null_i = ctypes.POINTER(ctypes.c_int)()
    rc = lib().orc_build_j(*args, _d(Dv), _d(J.view(np.float64)) if want_J else null_d, _d(energy),
                           _d(rho) if want_rho else null_d, _i(miller) if want_rho else null_i,
                           int(nG), ctypes.byref(nG_out), _d(grad) if want_grad else null_d,
                           int(nthreads), int(getattr(prob, "pair_gcut", 0) if pair_gcut is None else pair_gcut),
                           float(getattr(prob, "alpha_cut", 0.0) if alpha_cut is None else alpha_cut))
    if rc != 0:
        raise RuntimeError(f"oracle failed ({rc})")
    out = OracleResult(E_real=energy[0], E_G=energy[1], E_k=energy[2], maxImJ=energy[3],
                       maxJ=energy[4], charge=energy[5], nG=nG_out.value)
    if want_J:
        out["J"] = J
    if want_rho:
        out["rho"] = rho[:nG, 0] + 1j * rho[:nG, 1]
        out["miller"] = miller[:nG].copy()
    if want_grad:
        out["grad"] = grad
    return out


def pair_cut(la, lb, aa, RA, ab, RB, omega, eps_G, G):
    """(screening objective at |G| = G, cut radius) of one normalised primitive pair."""
    out = np.zeros(2)
    lib().orc_pair_cut(int(la), int(lb), float(aa), _d(np.ascontiguousarray(RA, dtype=np.float64)), float(ab),
                       _d(np.ascontiguousarray(RB, dtype=np.float64)), float(omega), float(eps_G), float(G),
                       _d(out))
    return float(out[0]), float(out[1])


def ft_axis(i, j, aa, Ax, ab, Bx, G):
    out = np.zeros(2)
    lib().orc_ft_axis(int(i), int(j), float(aa), float(Ax), float(ab), float(Bx), float(G), _d(out))
    return complex(out[0], out[1])


def pair_ft(la, lb, aa, RA, ab, RB, G, deriv=False):
    """Normalised Cartesian block [ncart(la)][ncart(lb)] (unit coefficients)."""
    nca, ncb = (la + 1) * (la + 2) // 2, (lb + 1) * (lb + 2) // 2
    RA = np.ascontiguousarray(RA, dtype=np.float64)
    RB = np.ascontiguousarray(RB, dtype=np.float64)
    G = np.ascontiguousarray(G, dtype=np.float64)
    out = np.zeros((nca, ncb, 2))
    null_d = ctypes.POINTER(ctypes.c_double)()
    if deriv:
        dA = np.zeros((3, nca, ncb, 2))
        dB = np.zeros((3, nca, ncb, 2))
        lib().orc_pair_ft(int(la), int(lb), float(aa), _d(RA), float(ab), _d(RB), _d(G), _d(out),
                          _d(dA), _d(dB))
        return (out[..., 0] + 1j * out[..., 1], dA[..., 0] + 1j * dA[..., 1],
                dB[..., 0] + 1j * dB[..., 1])
    lib().orc_pair_ft(int(la), int(lb), float(aa), _d(RA), float(ab), _d(RB), _d(G), _d(out),
                      null_d, null_d)
    return out[..., 0] + 1j * out[..., 1]
