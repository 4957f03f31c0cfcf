"""FP64 CPU oracle for the CRKSPH neighbour passes (test infrastructure).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark
import this package. The GPU library never does, and this package never
imports the library: the two share nothing but the seeded inputs.

The arithmetic lives in ``crk_oracle.c`` (plain C, FP64, built with
-ffp-contract=off, OpenMP over particles); this module loads it with ctypes
and wraps each pass. ``hnet.py`` holds the NumPy FP64 oracle of the
smoothing-length network.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "crk_oracle.c")
_LIB = os.path.join(_HERE, "liborc.so")

_d = C.c_double
_i64 = C.c_int64
_int = C.c_int
_p = C.c_void_p


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (FP64, no contraction, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(_LIB)
        L.orc_threads.restype = _int
        L.orc_threads.argtypes = []
        L.orc_W.restype = _d
        L.orc_W.argtypes = [_d, _d]
        L.orc_dWdr.restype = _d
        L.orc_dWdr.argtypes = [_d, _d]
        L.orc_kernel_eval.argtypes = [_i64, _p, _p, _p, _p]
        L.orc_neighbors_brute.restype = _i64
        L.orc_neighbors_brute.argtypes = [_i64, _p, _p, _p, _p, _d, _int, _int, _p, _p]
        L.orc_neighbors_grid.restype = _i64
        L.orc_neighbors_grid.argtypes = [_i64, _p, _p, _p, _p, _d, _int, _p, _p]
        L.orc_volume.argtypes = [_i64, _p, _p, _p, _p, _d, _int, _p, _p, _p, _p, _p]
        L.orc_nsum_at.restype = _d
        L.orc_nsum_at.argtypes = [_i64, _p, _p, _p, _d, _int, _i64, _d]
        L.orc_moments.argtypes = [_i64, _p, _p, _p, _p, _p, _d, _int, _p, _p] + [_p] * 6
        L.orc_corrections.restype = _i64
        L.orc_corrections.argtypes = [_i64] + [_p] * 11
        L.orc_rk_pairs.argtypes = [_i64, _p, _p, _p, _p, _d, _int, _p, _p, _p, _p, _i64,
                                   _p, _p, _p, _p, _p]
        L.orc_gradv.argtypes = [_i64, _p, _p, _p, _p, _d, _int, _p, _p, _p, _p, _p, _p, _p, _p, _p]
        L.orc_limiter.restype = _d
        L.orc_limiter.argtypes = [_d, _d, _d, _d, _d]
        L.orc_derivatives.argtypes = [_i64, _p, _p, _p, _p, _d, _int] + [_p] * 18
        L.orc_compatible_energy.argtypes = [_i64, _p, _p, _p, _p, _d, _int] + [_p] * 15 + [_d, _p]
        L.orc_compatible_energy.restype = None
        L.orc_thacker_step.restype = _d
        L.orc_thacker_step.argtypes = [_d, _d, _d]
        L.orc_hnet_features.argtypes = [_i64, _p, _p, _p, _p, _d, _d, _p]
        L.orc_hsolve.restype = _i64
        L.orc_hsolve.argtypes = [_i64, _p, _p, _p, _d, _int, _d, _d, _int, _p, _p]
        L.orc_rows_for.restype = _i64
        L.orc_rows_for.argtypes = [_i64, _p, _p, _p, _p, _d, _int, _i64, _p, _p, _p, _i64]
        L.orc_hsolve_for.restype = _i64
        L.orc_hsolve_for.argtypes = [_i64, _p, _p, _p, _d, _p, _d, _d, _int, _i64, _p, _p, _p, _p]
        _lib = L
    return _lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a):
    return None if a is None else a.ctypes.data_as(_p)


def threads() -> int:
    """OpenMP threads the oracle's loops run on."""
    return int(lib().orc_threads())


# ---------------------------------------------------------------- kernel
def W(r, H):
    r = _f64(np.broadcast_to(r, np.broadcast(r, H).shape))
    H = _f64(np.broadcast_to(H, r.shape))
    w = np.empty_like(r)
    dw = np.empty_like(r)
    lib().orc_kernel_eval(r.size, _ptr(r), _ptr(H), _ptr(w), _ptr(dw))
    return w


def dWdr(r, H):
    r = _f64(np.broadcast_to(r, np.broadcast(r, H).shape))
    H = _f64(np.broadcast_to(H, r.shape))
    w = np.empty_like(r)
    dw = np.empty_like(r)
    lib().orc_kernel_eval(r.size, _ptr(r), _ptr(H), _ptr(w), _ptr(dw))
    return dw


# ------------------------------------------------------------ neighbours
def neighbors(x, y, z, H, L=1.0, periodic=True, which=0, method="auto"):
    """CSR (offsets int64 [n+1], idx int32) of N_g (which=0, self included)
    or N_s (which=1), rows ascending."""
    x, y, z, H = map(_f64, (x, y, z, H))
    n = x.shape[0]
    off = np.zeros(n + 1, dtype=np.int64)
    if method == "auto":
        method = "brute" if (n <= 4096 or not periodic) else "grid"
    if method == "brute":
        tot = lib().orc_neighbors_brute(n, _ptr(x), _ptr(y), _ptr(z), _ptr(H), L, int(periodic),
                                        which, _ptr(off), None)
        idx = np.empty(tot, dtype=np.int32)
        lib().orc_neighbors_brute(n, _ptr(x), _ptr(y), _ptr(z), _ptr(H), L, int(periodic), which,
                                  _ptr(off), _ptr(idx))
    else:
        if not periodic:
            raise ValueError("the grid search is for periodic boxes")
        tot = lib().orc_neighbors_grid(n, _ptr(x), _ptr(y), _ptr(z), _ptr(H), L, which,
                                       _ptr(off), None)
        idx = np.empty(tot, dtype=np.int32)
        lib().orc_neighbors_grid(n, _ptr(x), _ptr(y), _ptr(z), _ptr(H), L, which, _ptr(off),
                                 _ptr(idx))
    return off, idx


# ----------------------------------------------------------------- passes
def volume(x, y, z, H, goff, gidx, L=1.0, periodic=True):
    x, y, z, H = map(_f64, (x, y, z, H))
    n = x.shape[0]
    nsum, V, N = np.empty(n), np.empty(n), np.empty(n)
    lib().orc_volume(n, _ptr(x), _ptr(y), _ptr(z), _ptr(H), L, int(periodic), _ptr(goff),
                     _ptr(gidx), _ptr(nsum), _ptr(V), _ptr(N))
    return nsum, V, N


def nsum_at(x, y, z, i, Hi, L=1.0, periodic=True):
    x, y, z = map(_f64, (x, y, z))
    return lib().orc_nsum_at(x.shape[0], _ptr(x), _ptr(y), _ptr(z), L, int(periodic), int(i),
                             float(Hi))


def moments(x, y, z, H, V, goff, gidx, L=1.0, periodic=True):
    """dict of m0 [n], m1 [3,n], m2 [6,n], gm0 [3,n], gm1 [9,n], gm2 [18,n]."""
    x, y, z, H, V = map(_f64, (x, y, z, H, V))
    n = x.shape[0]
    out = dict(m0=np.empty(n), m1=np.empty((3, n)), m2=np.empty((6, n)), gm0=np.empty((3, n)),
               gm1=np.empty((9, n)), gm2=np.empty((18, n)))
    lib().orc_moments(n, _ptr(x), _ptr(y), _ptr(z), _ptr(H), _ptr(V), L, int(periodic),
                      _ptr(goff), _ptr(gidx), *[_ptr(out[k]) for k in
                                                ("m0", "m1", "m2", "gm0", "gm1", "gm2")])
    return out


def corrections(mom):
    """dict of A [n], B [3,n], gA [3,n], gB [9,n], singular [n] int32, n_singular."""
    n = mom["m0"].shape[0]
    src = [_f64(mom[k]) for k in ("m0", "m1", "m2", "gm0", "gm1", "gm2")]
    out = dict(A=np.empty(n), B=np.empty((3, n)), gA=np.empty((3, n)), gB=np.empty((9, n)),
               singular=np.empty(n, dtype=np.int32))
    ns = lib().orc_corrections(n, *[_ptr(a) for a in src],
                               *[_ptr(out[k]) for k in ("A", "B", "gA", "gB", "singular")])
    out["n_singular"] = int(ns)
    return out


def rk_pairs(x, y, z, H, corr, pi, pj, L=1.0, periodic=True):
    """W^R_ij, grad W^R_ij [3,npair] and d_ij [3,npair] for ordered pairs (pi, pj)."""
    x, y, z, H = map(_f64, (x, y, z, H))
    pi = np.ascontiguousarray(pi, dtype=np.int32)
    pj = np.ascontiguousarray(pj, dtype=np.int32)
    npair = pi.shape[0]
    WR, GR, d = np.empty(npair), np.empty((3, npair)), np.empty((3, npair))
    c = [_f64(corr[k]) for k in ("A", "B", "gA", "gB")]
    lib().orc_rk_pairs(x.shape[0], _ptr(x), _ptr(y), _ptr(z), _ptr(H), L, int(periodic),
                       *[_ptr(a) for a in c], npair, _ptr(pi), _ptr(pj), _ptr(WR), _ptr(GR),
                       _ptr(d))
    return WR, GR, d


def gradv(x, y, z, H, v, V, corr, goff, gidx, L=1.0, periodic=True):
    x, y, z, H, v, V = map(_f64, (x, y, z, H, v, V))
    n = x.shape[0]
    out = np.empty((9, n))
    c = [_f64(corr[k]) for k in ("A", "B", "gA", "gB")]
    lib().orc_gradv(n, _ptr(x), _ptr(y), _ptr(z), _ptr(H), L, int(periodic), _ptr(v), _ptr(V),
                    *[_ptr(a) for a in c], _ptr(goff), _ptr(gidx), _ptr(out))
    return out


def limiter(si, sj, eta, eta_c, eta_f):
    return lib().orc_limiter(float(si), float(sj), float(eta), float(eta_c), float(eta_f))


PARAM_KEYS = ("gamma", "Cl", "Cq", "eps", "nh", "eta_c", "eta_f", "a", "adot")


def params(nres: float = 64.0, **over) -> dict:
    """Solver parameters. n_h follows from the target neighbour count by
    N_res = (4 pi / 3) n_h^3 (n_h = 4 <-> N_res = 268, Sec. 3.6), and the
    limiter scales are (1/n_h, 0.2/n_h); the viscosity constants are
    (C_l, C_q) = (2, 1) and eps = 0.1 (Sec. 2.2)."""
    nh = (3.0 * nres / (4.0 * math.pi)) ** (1.0 / 3.0)
    p = dict(gamma=5.0 / 3.0, Cl=2.0, Cq=1.0, eps=0.1, nh=nh, eta_c=1.0 / nh, eta_f=0.2 / nh,
             a=1.0, adot=0.0)
    p.update(over)
    return p


def derivatives(x, y, z, H, v, m, u, rho, V, corr, gv, soff, sidx, prm, L=1.0, periodic=True,
                ts=None):
    """(dp/dt [3,n], du/dt [n], SF [n], SE [n]); with a dict ``ts`` also the
    time-step terms ts["vsig"] (closing speed, max over the pair set) and
    ts["qrho"] (max over the pairs of Q_i / rho_i)."""
    x, y, z, H, v, m, u, V, gv = map(_f64, (x, y, z, H, v, m, u, V, gv))
    rho = None if rho is None else _f64(rho)
    n = x.shape[0]
    dv, du, SF, SE = np.empty((3, n)), np.empty(n), np.empty(n), np.empty(n)
    VS, QR = (np.empty(n), np.empty(n)) if ts is not None else (None, None)
    c = [_f64(corr[k]) for k in ("A", "B", "gA", "gB")]
    pa = np.array([prm[k] for k in PARAM_KEYS], dtype=np.float64)
    lib().orc_derivatives(n, _ptr(x), _ptr(y), _ptr(z), _ptr(H), L, int(periodic), _ptr(v),
                          _ptr(m), _ptr(u), _ptr(rho), _ptr(V), *[_ptr(a) for a in c], _ptr(gv),
                          _ptr(pa), _ptr(soff), _ptr(sidx), _ptr(dv), _ptr(du), _ptr(SF),
                          _ptr(SE), _ptr(VS), _ptr(QR))
    if ts is not None:
        ts["vsig"], ts["qrho"] = VS, QR
    return dv, du, SF, SE


def compatible_energy(x, y, z, H, v, m, u, rho, V, corr, gv, soff, sidx, prm, dpdt, dt, L=1.0,
                      periodic=True, pk=None):
    """Delta u [n] of the compatible energy update over the time step dt
    (eqs. compEng, compEng2, Eij, ptdt, fij), from the state the derivative
    pass saw and its dp/dt [3, n]; pk [3, n], when given, is the momentum at
    the start of the kick (else a v)."""
    x, y, z, H, v, m, u, V, gv, dpdt = map(_f64, (x, y, z, H, v, m, u, V, gv, dpdt))
    pk = None if pk is None else _f64(pk)
    rho = None if rho is None else _f64(rho)
    n = x.shape[0]
    du = np.empty(n)
    c = [_f64(corr[k]) for k in ("A", "B", "gA", "gB")]
    pa = np.array([prm[k] for k in PARAM_KEYS], dtype=np.float64)
    lib().orc_compatible_energy(n, _ptr(x), _ptr(y), _ptr(z), _ptr(H), L, int(periodic), _ptr(v),
                                _ptr(m), _ptr(u), _ptr(rho), _ptr(V), *[_ptr(a) for a in c],
                                _ptr(gv), _ptr(pa), _ptr(soff), _ptr(sidx), _ptr(dpdt), _ptr(pk),
                                float(dt), _ptr(du))
    return du


def timestep(H, u, m, rho, V, gv, vsig, qrho, prm, zeta=4.0, c_cfl=0.25):
    """Courant criterion of Sec. 3.1 per particle: (v_max [n], dt_hyd [n]) with
    v_max = max(v_sig, c_s, c_sq, (h_hat / a) |div u|), c_sq = sqrt(zeta Q/rho),
    |div u| = |Tr grad v + 3 adot|, h_hat = H / n_h, and dt_hyd = C_CFL h_hat /
    v_max in time (the caller applies dy/dt)."""
    H, u, m, V = map(_f64, (H, u, m, V))
    gv = _f64(gv).reshape(9, -1)
    rho = m / V if rho is None else _f64(rho)
    P = (prm["gamma"] - 1.0) * rho * u
    cs = np.sqrt(prm["gamma"] * P / rho)
    csq = np.sqrt(zeta * _f64(qrho))
    hh = H / prm["nh"]
    divu = np.abs(gv[0] + gv[4] + gv[8] + 3.0 * prm["adot"])
    vmax = np.maximum(np.maximum(_f64(vsig), cs), np.maximum(csq, hh / prm["a"] * divu))
    return vmax, c_cfl * hh / vmax


def time_levels(H, dt_hyd, dvdt, prm, r_soft, dt_sub, l_max):
    """Hierarchical time-step levels of Sec. 3.1 per particle, in time units:
    dt_acc = sqrt(min(h_hat, r_soft) / |a_hyd|) with the hydrodynamic
    acceleration a_hyd = dp/dt / a^2 (infinite where it vanishes; gravity is
    not part of these passes), dt_min = min(dt_hyd, dt_acc), and the level l,
    the smallest l >= 0 with dt_min > dt_sub / 2^l (l_max + 1 when none up
    to l_max qualifies). Returns (dt_acc, dt_min, level int32)."""
    H, dt_hyd, dvdt = _f64(H), _f64(dt_hyd), _f64(dvdt).reshape(3, -1)
    hh = H / prm["nh"]
    acc = np.sqrt((dvdt ** 2).sum(0)) / prm["a"] ** 2
    with np.errstate(divide="ignore"):
        dt_acc = np.where(acc > 0.0, np.sqrt(np.minimum(hh, r_soft) / np.where(acc > 0.0, acc, 1.0)),
                          np.inf)
    dt_min = np.minimum(dt_hyd, dt_acc)
    level = np.empty(H.shape[0], dtype=np.int32)
    for i in range(H.shape[0]):
        l = 0
        while l <= l_max and not dt_min[i] > dt_sub / 2.0 ** l:
            l += 1
        level[i] = l
    return dt_acc, dt_min, level


def thacker_step(H, N, Nres):
    return lib().orc_thacker_step(float(H), float(N), float(Nres))


def hsolve(x, y, z, H0, Nres, tol=1e-7, max_iter=100, L=1.0, periodic=True):
    """(H [n], iterations [n] int32, n_not_converged)."""
    x, y, z = map(_f64, (x, y, z))
    H = _f64(H0).copy()
    it = np.empty(x.shape[0], dtype=np.int32)
    nf = lib().orc_hsolve(x.shape[0], _ptr(x), _ptr(y), _ptr(z), L, int(periodic), float(Nres),
                          float(tol), int(max_iter), _ptr(H), _ptr(it))
    return H, it, int(nf)


def hnet_features(x, y, z, H, Nres, L=1.0):
    """[8, n] input features of the smoothing-length network at radius H."""
    x, y, z, H = map(_f64, (x, y, z, H))
    n = x.shape[0]
    out = np.empty((8, n))
    lib().orc_hnet_features(n, _ptr(x), _ptr(y), _ptr(z), _ptr(H), float(L), float(Nres), _ptr(out))
    return out


def pipeline(ps, prm, periodic=True, method="auto", dt=None):
    """Every pass in the paper's data order for one particle set:
    neighbour sets -> volume -> moments -> corrections -> grad v -> derivatives
    (-> the compatible energy update over dt, when dt is given).
    Returns a dict with every intermediate (original particle order)."""
    x, y, z, H = ps.x, ps.y, ps.z, ps.H
    L = ps.L
    goff, gidx = neighbors(x, y, z, H, L, periodic, 0, method)
    soff, sidx = neighbors(x, y, z, H, L, periodic, 1, method)
    nsum, V, N = volume(x, y, z, H, goff, gidx, L, periodic)
    mom = moments(x, y, z, H, V, goff, gidx, L, periodic)
    corr = corrections(mom)
    gv = gradv(x, y, z, H, ps.v, V, corr, goff, gidx, L, periodic)
    ts = {}
    dv, du, SF, SE = derivatives(x, y, z, H, ps.v, ps.m, ps.u, ps.rho, V, corr, gv, soff, sidx,
                                 prm, L, periodic, ts=ts)
    vmax, dt_hyd = timestep(H, ps.u, ps.m, ps.rho, V, gv, ts["vsig"], ts["qrho"], prm)
    out = dict(goff=goff, gidx=gidx, soff=soff, sidx=sidx, nsum=nsum, V=V, N=N, gradv=gv,
               dvdt=dv, dudt=du, SF=SF, SE=SE, n_pairs=int(soff[-1]), vsig=ts["vsig"],
               qrho=ts["qrho"], vmax=vmax, dt_hyd=dt_hyd)
    if dt is not None:
        out["du_compat"] = compatible_energy(x, y, z, H, ps.v, ps.m, ps.u, ps.rho, V, corr, gv, soff,
                                             sidx, prm, dv, dt, L, periodic)
    out.update(mom)
    out.update(corr)
    return out


# ------------------------------------------------------ velocity Verlet
def _compat_half(st, d, prm, k, pk, periodic):
    """Delta u of a half kick of length k with the pair forces of the
    evaluation d at state st, starting from the momenta pk."""
    return compatible_energy(st.x, st.y, st.z, st.H, st.v, st.m, st.u, st.rho, d["V"], d,
                             d["gradv"], d["soff"], d["sidx"], prm, d["dvdt"], k, st.L, periodic,
                             pk=pk)


def verlet_step(ps, prm, dt, d0=None, periodic=True, energy="eng"):
    """One step of the velocity-Verlet hydro operator, eq. verletOP, with the
    time step dt = (dt/dy) Delta y and a, adot held over the step. With
    p = a v and D = (dp/dt, du/dt) from the derivative pass (eqs. mom, eng):
      p^1/2 = p^0 + dt/2 dp/dt(0),      u^1/2 = u^0 + dt/2 du/dt(0),
      x^1   = x^0 + p^1/2 dt / a^2      (wrapped into [0, L) when periodic),
      p_p   = p^1/2 + dt/2 dp/dt(0),    u_p   = u^1/2 + dt/2 du/dt(0),
      D(1)  = D at (x^1, p_p, u_p) with the same H, m (and rho if given),
      p^1   = p^1/2 + dt/2 dp/dt(1),    u^1   = u^1/2 + dt/2 du/dt(1).
    With energy="compat" each half kick's energy change is instead the
    compatible update (eqs. compEng-fij) of that kick: the pair forces of
    the evaluation the kick uses, the momenta the kick starts from, length
    dt/2; the opening kick's change is carried as a rate in D["dudt_kick"]
    (taken for a next step of the same dt), which also predicts u_p.
    d0 is D at the start state (dict with dvdt, dudt, and dudt_kick for
    "compat"); None evaluates it. Returns (state, D(1)): state is a
    namespace like ps at the end of the step (v = p / a); D(1) is the
    derivative pass's output there."""
    from types import SimpleNamespace
    a = prm["a"]
    L = ps.L
    k = 0.5 * dt
    compat = energy == "compat"
    gam = getattr(ps, "gamma", prm["gamma"])
    if d0 is None:
        d0 = pipeline(ps, prm, periodic)
        if compat:
            st0 = SimpleNamespace(x=ps.x, y=ps.y, z=ps.z, H=ps.H, m=ps.m, u=ps.u, v=ps.v,
                                  rho=ps.rho, L=L)
            d0["dudt_kick"] = _compat_half(st0, d0, prm, k, a * np.asarray(ps.v), periodic) / k
    rate0 = d0["dudt_kick"] if compat else d0["dudt"]
    c = dt / (a * a)
    ph = a * np.asarray(ps.v, dtype=np.float64) + k * d0["dvdt"]
    uh = np.asarray(ps.u, dtype=np.float64) + k * rate0
    x1 = []
    for q, comp in ((ps.x, 0), (ps.y, 1), (ps.z, 2)):
        xn = np.asarray(q, dtype=np.float64) + ph[comp] * c
        if periodic:
            xn = np.where(xn < 0.0, xn + L, xn)
            xn = np.where(xn >= L, xn - L, xn)
        x1.append(xn)
    pp = ph + k * d0["dvdt"]
    up = uh + k * rate0
    mid = SimpleNamespace(x=x1[0], y=x1[1], z=x1[2], H=ps.H, m=ps.m, u=up, v=pp / a,
                          rho=ps.rho, L=L, gamma=gam)
    d1 = pipeline(mid, prm, periodic)
    p1 = ph + k * d1["dvdt"]
    if compat:
        u1 = uh + _compat_half(mid, d1, prm, k, ph, periodic)
        d1["dudt_kick"] = _compat_half(mid, d1, prm, k, p1, periodic) / k
    else:
        u1 = uh + k * d1["dudt"]
    end = SimpleNamespace(x=x1[0], y=x1[1], z=x1[2], H=ps.H, m=ps.m, u=u1, v=p1 / a,
                          rho=ps.rho, L=L, gamma=gam)
    return end, d1


# ------------------------------------------------------ sampled evaluation
def rows_for(x, y, z, H, which, targets, L=1.0):
    """CSR rows of N_g (which 0, self included) or N_s (which 1) for the
    listed particles only, over the whole periodic set; rows ascending."""
    x, y, z, H = map(_f64, (x, y, z, H))
    t = np.ascontiguousarray(targets, dtype=np.int64)
    off = np.zeros(t.shape[0] + 1, dtype=np.int64)
    args = (x.shape[0], _ptr(x), _ptr(y), _ptr(z), _ptr(H), float(L), int(which), t.shape[0], _ptr(t),
            _ptr(off))
    tot = lib().orc_rows_for(*args, None, 0)
    idx = np.empty(max(tot, 1), dtype=np.int32)
    lib().orc_rows_for(*args, _ptr(idx), tot)
    return off, idx[:tot]


def hsolve_for(x, y, z, targets, H0, Nres, tol=1e-7, max_iter=100, L=1.0, H_grid=None):
    """The iteration of ``hsolve`` for the listed particles only, over every
    position. H0: starting radii of the targets. H_grid (all particles) only
    sizes the search grid. Returns (H, iterations, n_not_converged)."""
    x, y, z = map(_f64, (x, y, z))
    t = np.ascontiguousarray(targets, dtype=np.int64)
    H0 = _f64(H0)
    Hg = _f64(H_grid) if H_grid is not None else np.full(x.shape[0], float(np.mean(H0)))
    H = np.empty(t.shape[0])
    it = np.empty(t.shape[0], dtype=np.int32)
    nf = lib().orc_hsolve_for(x.shape[0], _ptr(x), _ptr(y), _ptr(z), float(L), _ptr(Hg), float(Nres),
                              float(tol), int(max_iter), t.shape[0], _ptr(t), _ptr(H0), _ptr(H),
                              _ptr(it))
    return H, it, int(nf)


def _sub_rows(S, owners, off, idx):
    """CSR over the sorted index set S: the rows of `owners` (sorted, a subset
    of S, row data off/idx in original indices) remapped into S, empty rows
    for the rest of S."""
    lens = np.zeros(S.shape[0], dtype=np.int64)
    lens[np.searchsorted(S, owners)] = np.diff(off)
    o = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    return o, np.searchsorted(S, idx).astype(np.int32)


def spot_check(ps, targets, prm, H=None):
    """Every pass for the listed particles only, exactly as ``pipeline``
    computes it on the whole set: the targets' pair sets (1-hop ring R1),
    the gather sets of R1 (2-hop ring R2) and those of R2 (R3) are found over
    all particles; volumes are evaluated on R2, moments, corrections and
    grad v on R1, and the derivatives on the targets, each with the same
    rows (ascending) as the whole-set oracle. Returns a dict of the outputs
    of ``pipeline`` at the sorted unique targets (key "targets")."""
    x, y, z = map(_f64, (ps.x, ps.y, ps.z))
    H = _f64(ps.H if H is None else H)
    L = ps.L
    T = np.unique(np.asarray(targets, dtype=np.int64))
    soff, sidx = rows_for(x, y, z, H, 1, T, L)
    R1 = np.union1d(T, sidx)
    g1off, g1idx = rows_for(x, y, z, H, 0, R1, L)
    R2 = np.union1d(R1, g1idx)
    g2off, g2idx = rows_for(x, y, z, H, 0, R2, L)
    R3 = np.union1d(R2, g2idx)
    # volumes on R2, over the positions of R3
    oA, iA = _sub_rows(R3, R2, g2off, g2idx)
    _, VA, NA = volume(x[R3], y[R3], z[R3], H[R3], oA, iA, L)
    pB = np.searchsorted(R3, R2)
    V2 = VA[pB]
    # moments, corrections and grad v on R1, over R2
    oB, iB = _sub_rows(R2, R1, g1off, g1idx)
    xb, yb, zb, hb = x[R2], y[R2], z[R2], H[R2]
    with np.errstate(all="ignore"):
        mom = moments(xb, yb, zb, hb, V2, oB, iB, L)
        corr = corrections(mom)
        gv = gradv(xb, yb, zb, hb, ps.v[:, R2], V2, corr, oB, iB, L)
    # derivatives on the targets, over R1
    pC = np.searchsorted(R2, R1)
    oC, iC = _sub_rows(R1, T, soff, sidx)
    cC = {k: corr[k][..., pC] for k in ("A", "B", "gA", "gB")}
    rho = None if ps.rho is None else _f64(ps.rho)[R1]
    dv, du, SF, SE = derivatives(x[R1], y[R1], z[R1], H[R1], ps.v[:, R1], _f64(ps.m)[R1],
                                 _f64(ps.u)[R1], rho, V2[pC], cC, gv[:, pC], oC, iC, prm, L)
    pT1 = np.searchsorted(R1, T)          # targets within R1
    pT2 = pC[pT1]                          # targets within R2
    out = dict(targets=T, V=V2[pT2], N=NA[np.searchsorted(R3, T)], gradv=gv[:, pT2],
               dvdt=dv[:, pT1], dudt=du[pT1], SF=SF[pT1], SE=SE[pT1],
               n_pairs=int(soff[-1]), rings=(T.shape[0], R1.shape[0], R2.shape[0], R3.shape[0]))
    for k, a in mom.items():
        out[k] = a[..., pT2]
    for k in ("A", "B", "gA", "gB", "singular"):
        out[k] = corr[k][..., pT2]
    return out
