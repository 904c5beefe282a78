"""ctypes front end of the FP64 CPU oracle (test infrastructure only).

Wraps oracle/liboracle.so (plain C, FP64) and adds the closed-form checks
written directly from their mathematical definitions.  Nothing here imports
or calls the product library.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)


class OrGrid(C.Structure):
    _fields_ = [("ndim", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32),
                ("nz", C.c_int32), ("npml", C.c_int32), ("nt", C.c_int32),
                ("dx", C.c_double), ("dt", C.c_double), ("pml_R", C.c_double),
                ("pml_vmax", C.c_double), ("f0_pml", C.c_double)]


def lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(HERE, "liboracle.so")
        if not os.path.exists(path):
            from . import build as _b
            _b.build()
        _LIB = C.CDLL(path)
    return _LIB


def grid(ndim=2, nx=1, ny=1, nz=1, npml=0, nt=1, dx=10.0, dt=1e-3,
         pml_R=1e-3, pml_vmax=3000.0, f0_pml=10.0):
    return OrGrid(ndim, nx, ny, nz, npml, nt, dx, dt, pml_R, pml_vmax, f0_pml)


def _d(a):
    return a.ctypes.data_as(_dp)


def _i(a):
    return a.ctypes.data_as(_ip)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def ricker(f0, t0, dt, nt):
    out = np.zeros(nt)
    lib().or_ricker(C.c_double(f0), C.c_double(t0), C.c_double(dt), C.c_int32(nt), _d(out))
    return out


def stencil_weights():
    l8, d8, s4 = np.zeros(5), np.zeros(5), np.zeros(2)
    lib().or_stencil_weights(_d(l8), _d(d8), _d(s4))
    return l8, d8, s4


# ---------------------------------------------------------------- acoustic 2-D
def ac2_pad(g, c):
    P = g.npml
    NX, NZ = g.nx + 2 * P, g.nz + 2 * P
    cp, zx, zz = np.zeros((NZ, NX)), np.zeros(NX), np.zeros(NZ)
    lib().or_ac2_pad(C.byref(g), _d(_f64(c)), _d(cp), _d(zx), _d(zz))
    return cp, zx, zz


def ac2_step(g, c_pad, X, src_idx=-1, src_val=0.0):
    """X = (u, um, px, pz) padded arrays -> (Y tuple, w)."""
    X = [_f64(x) for x in X]
    Y = [np.zeros_like(X[0]) for _ in range(4)]
    w = np.zeros_like(X[0])
    lib().or_ac2_step(C.byref(g), _d(_f64(c_pad)), _d(X[0]), _d(X[1]), _d(X[2]), _d(X[3]),
                      C.c_int64(src_idx), C.c_double(src_val),
                      _d(Y[0]), _d(Y[1]), _d(Y[2]), _d(Y[3]), _d(w))
    return Y, w


def ac2_step_T(g, c_pad, X, aY, src_idx=-1):
    X = [_f64(x) for x in X]
    aY = [_f64(x) for x in aY]
    aX = [np.zeros_like(X[0]) for _ in range(4)]
    gC = np.zeros_like(X[0])
    sb = C.c_double(0.0)
    lib().or_ac2_step_T(C.byref(g), _d(_f64(c_pad)), _d(X[0]), _d(X[2]), _d(X[3]),
                        _d(aY[0]), _d(aY[1]), _d(aY[2]), _d(aY[3]),
                        _d(aX[0]), _d(aX[1]), _d(aX[2]), _d(aX[3]), _d(gC),
                        C.c_int64(src_idx), C.byref(sb))
    return aX, gC, sb.value


def ac2_forward(g, c, src, wav, rec):
    src, rec, wav = _i32(src), _i32(rec), _f64(wav)
    ns, nrec = src.shape[0], rec.shape[1]
    seis = np.zeros((ns, g.nt, nrec))
    rc = lib().or_ac2_forward(C.byref(g), _d(_f64(c)), C.c_int32(ns), _i(src), _d(wav),
                              C.c_int32(nrec), _i(rec), _d(seis))
    if rc:
        raise ValueError("oracle: invalid geometry or grid")
    return seis


def ac2_gradient(g, c, src, wav, rec, dJdd, ckpt=0, want_wav=False):
    src, rec, wav = _i32(src), _i32(rec), _f64(wav)
    ns, nrec = src.shape[0], rec.shape[1]
    seis = np.zeros((ns, g.nt, nrec))
    grad = np.zeros((g.nz, g.nx))
    gw = np.zeros((ns, g.nt)) if want_wav else None
    rc = lib().or_ac2_gradient(C.byref(g), _d(_f64(c)), C.c_int32(ns), _i(src), _d(wav),
                               C.c_int32(nrec), _i(rec), _d(_f64(dJdd)), C.c_int32(ckpt),
                               _d(grad), _d(seis), _d(gw) if want_wav else None)
    if rc:
        raise ValueError("oracle: invalid geometry or grid")
    return (grad, seis, gw) if want_wav else (grad, seis)


def ac2_forward_ms(g, c, src, wav, rec):
    """Several source cells per shot: src [ns][nsrc][2], wav [ns][nsrc][nt]."""
    src, rec, wav = _i32(src), _i32(rec), _f64(wav)
    ns, nsrc, nrec = src.shape[0], src.shape[1], rec.shape[1]
    seis = np.zeros((ns, g.nt, nrec))
    rc = lib().or_ac2_forward_ms(C.byref(g), _d(_f64(c)), C.c_int32(ns), C.c_int32(nsrc), _i(src), _d(wav),
                                 C.c_int32(nrec), _i(rec), _d(seis))
    if rc:
        raise ValueError("oracle: invalid geometry or grid")
    return seis


def ac2_gradient_ms(g, c, src, wav, rec, dJdd, ckpt=0):
    """(dJ/dc, seismograms, dJ/dwav [ns][nsrc][nt]) for several source cells per shot."""
    src, rec, wav = _i32(src), _i32(rec), _f64(wav)
    ns, nsrc, nrec = src.shape[0], src.shape[1], rec.shape[1]
    seis = np.zeros((ns, g.nt, nrec))
    grad = np.zeros((g.nz, g.nx))
    gw = np.zeros((ns, nsrc, g.nt))
    rc = lib().or_ac2_gradient_ms(C.byref(g), _d(_f64(c)), C.c_int32(ns), C.c_int32(nsrc), _i(src), _d(wav),
                                  C.c_int32(nrec), _i(rec), _d(_f64(dJdd)), C.c_int32(ckpt),
                                  _d(grad), _d(seis), _d(gw))
    if rc:
        raise ValueError("oracle: invalid geometry or grid")
    return grad, seis, gw


# ------------------------------------------------ acoustic 2-D, divergence form
def ad2_coefficients(g, c):
    """Half-node coefficients (kx, kz) of the padded model, each (NZ, NX)."""
    P = g.npml
    kx, kz = np.zeros((g.nz + 2 * P, g.nx + 2 * P)), np.zeros((g.nz + 2 * P, g.nx + 2 * P))
    lib().or_ad2_coefficients(C.byref(g), _d(_f64(c)), _d(kx), _d(kz))
    return kx, kz


def ad2_step(g, c, X, src_idx=-1, src_val=0.0):
    """X: (6, NZ, NX) state (u, um, psix, psiz, xix, xiz) -> next state."""
    X = _f64(X)
    Y = np.zeros_like(X)
    lib().or_ad2_step(C.byref(g), _d(_f64(c)), _d(X), C.c_int64(src_idx), C.c_double(src_val), _d(Y))
    return Y


def ad2_step_T(g, c, X, aY):
    """Transpose of the step at state X: (aX, dJ/dkx, dJ/dkz)."""
    X, aY = _f64(X), _f64(aY)
    aX = np.zeros_like(X)
    gkx, gkz = np.zeros_like(X[0]), np.zeros_like(X[0])
    lib().or_ad2_step_T(C.byref(g), _d(_f64(c)), _d(X), _d(aY), _d(aX), _d(gkx), _d(gkz))
    return aX, gkx, gkz


def _ad2_geom(src, rec, wav):
    src, rec, wav = _i32(src), _i32(rec), _f64(wav)
    if src.ndim == 2:                       # one node per shot
        src, wav = src[:, None], wav[:, None]
    return src, rec, wav


def ad2_forward(g, c, src, wav, rec):
    """src [ns][nsrc][2] (or [ns][2]), wav [ns][nsrc][nt] (or [ns][nt]) -> seis [ns][nt][nrec]."""
    src, rec, wav = _ad2_geom(src, rec, wav)
    ns, nsrc, nrec = src.shape[0], src.shape[1], rec.shape[1]
    seis = np.zeros((ns, g.nt, nrec))
    rc = lib().or_ad2_forward(C.byref(g), _d(_f64(c)), C.c_int32(ns), C.c_int32(nsrc), _i(src), _d(wav),
                              C.c_int32(nrec), _i(rec), _d(seis))
    if rc:
        raise ValueError("oracle: invalid geometry or grid")
    return seis


def ad2_gradient(g, c, src, wav, rec, dJdd, ckpt=0):
    """(dJ/dc, seismograms, dJ/dwav [ns][nsrc][nt])."""
    src, rec, wav = _ad2_geom(src, rec, wav)
    ns, nsrc, nrec = src.shape[0], src.shape[1], rec.shape[1]
    seis = np.zeros((ns, g.nt, nrec))
    grad = np.zeros((g.nz, g.nx))
    gw = np.zeros((ns, nsrc, g.nt))
    rc = lib().or_ad2_gradient(C.byref(g), _d(_f64(c)), C.c_int32(ns), C.c_int32(nsrc), _i(src), _d(wav),
                               C.c_int32(nrec), _i(rec), _d(_f64(dJdd)), C.c_int32(ckpt),
                               _d(grad), _d(seis), _d(gw))
    if rc:
        raise ValueError("oracle: invalid geometry or grid")
    return grad, seis, gw


def misfit(pred, obs):
    pred, obs = _f64(pred), _f64(obs)
    r = np.zeros_like(pred)
    lib().or_misfit.restype = C.c_double
    J = lib().or_misfit(_d(pred), _d(obs), C.c_int64(pred.size), _d(r))
    return J, r


# ------------------------------------------------- closed-form 2-D Green's function
def greens2d_ricker(r, c, t, f0, t0, nq=4000):
    """Pressure of u_tt = c^2 lap u + delta(x) s(t) in an infinite 2-D medium
    at distance r, for s = Ricker(f0, t0):

        u(r, t) = 1/(2 pi c^2) * int_0^{acosh(ct/r)} s(t - (r/c) cosh(eta)) d eta

    (the 2-D Green's function H(ct - r) / (2 pi c sqrt(c^2 t^2 - r^2))
    convolved with s, after the substitution c(t - tau) = r cosh(eta)).
    Evaluated with nq-point Gauss-Legendre quadrature per time sample."""
    t = np.asarray(t, dtype=np.float64)
    out = np.zeros_like(t)
    xg, wg = np.polynomial.legendre.leggauss(nq)
    for i, ti in enumerate(t):
        if c * ti <= r:
            continue
        top = np.arccosh(c * ti / r)
        eta = 0.5 * top * (xg + 1.0)
        tau = ti - (r / c) * np.cosh(eta)
        a = (np.pi * f0 * (tau - t0)) ** 2
        s = (1.0 - 2.0 * a) * np.exp(-a)
        out[i] = 0.5 * top * np.dot(wg, s) / (2.0 * np.pi * c * c)
    return out


# ---------------------------------------------------------------- acoustic 3-D
def _ptrs(arrs):
    arr_t = _dp * len(arrs)
    return arr_t(*[_d(a) for a in arrs])


def ac3_pad(g, c):
    P = g.npml
    sh = (g.nz + 2 * P, g.ny + 2 * P, g.nx + 2 * P)
    cp = np.zeros(sh)
    zx, zy, zz = np.zeros(sh[2]), np.zeros(sh[1]), np.zeros(sh[0])
    lib().or_ac3_pad(C.byref(g), _d(_f64(c)), _d(cp), _d(zx), _d(zy), _d(zz))
    return cp, zx, zy, zz


def ac3_step(g, c_pad, X, src_idx=-1, src_val=0.0):
    """X = (u, um, phix, phiy, phiz, psi) padded arrays -> (Y list, w)."""
    X = [_f64(x) for x in X]
    Y = [np.zeros_like(X[0]) for _ in range(6)]
    w = np.zeros_like(X[0])
    lib().or_ac3_step(C.byref(g), _d(_f64(c_pad)), _ptrs(X), C.c_int64(src_idx), C.c_double(src_val),
                      _ptrs(Y), _d(w))
    return Y, w


def ac3_step_T(g, c_pad, X, aY, src_idx=-1):
    X = [_f64(x) for x in X]
    aY = [_f64(x) for x in aY]
    aX = [np.zeros_like(X[0]) for _ in range(6)]
    gC = np.zeros_like(X[0])
    sb = C.c_double(0.0)
    lib().or_ac3_step_T(C.byref(g), _d(_f64(c_pad)), _ptrs(X), _ptrs(aY), _ptrs(aX), _d(gC),
                        C.c_int64(src_idx), C.byref(sb))
    return aX, gC, sb.value


def ac3_forward(g, c, src, wav, rec):
    src, rec, wav = _i32(src), _i32(rec), _f64(wav)
    ns, nrec = src.shape[0], rec.shape[1]
    seis = np.zeros((ns, g.nt, nrec))
    if lib().or_ac3_forward(C.byref(g), _d(_f64(c)), C.c_int32(ns), _i(src), _d(wav),
                            C.c_int32(nrec), _i(rec), _d(seis)):
        raise ValueError("oracle: invalid geometry or grid")
    return seis


def ac3_gradient(g, c, src, wav, rec, dJdd, ckpt=0, want_wav=False):
    src, rec, wav = _i32(src), _i32(rec), _f64(wav)
    ns, nrec = src.shape[0], rec.shape[1]
    seis = np.zeros((ns, g.nt, nrec))
    grad = np.zeros((g.nz, g.ny, g.nx))
    gw = np.zeros((ns, g.nt)) if want_wav else None
    if lib().or_ac3_gradient(C.byref(g), _d(_f64(c)), C.c_int32(ns), _i(src), _d(wav),
                             C.c_int32(nrec), _i(rec), _d(_f64(dJdd)), C.c_int32(ckpt),
                             _d(grad), _d(seis), _d(gw) if want_wav else None):
        raise ValueError("oracle: invalid geometry or grid")
    return (grad, seis, gw) if want_wav else (grad, seis)


def greens3d_ricker(r, c, t, f0, t0):
    """u_tt = c^2 lap u + delta(x) s(t) in infinite 3-D space:
    u(r, t) = s(t - r/c) / (4 pi c^2 r)."""
    tau = np.asarray(t, dtype=np.float64) - r / c
    a = (np.pi * f0 * (tau - t0)) ** 2
    s = np.where(tau >= 0, (1.0 - 2.0 * a) * np.exp(-a), 0.0)
    return s / (4.0 * np.pi * c * c * r)


# ---------------------------------------------------------------- elastic 2-D
def cpml_profile(g, n, half):
    """CPML (a, b) of the oracle at every padded position i + half/2 of an axis
    with n physical cells (half = 0: integer nodes, 1: half nodes)."""
    P = g.npml
    a, b = np.zeros(n + 2 * P), np.zeros(n + 2 * P)
    fa, fb = C.c_double(0.0), C.c_double(0.0)
    f = lib().or_cpml_at
    f.argtypes = [C.POINTER(OrGrid), C.c_int, C.c_double, _dp, _dp]
    for i in range(n + 2 * P):
        f(C.byref(g), n, i + 0.5 * half, C.byref(fa), C.byref(fb))
        a[i], b[i] = fa.value, fb.value
    return a, b


EL2_FIELDS = ("vx", "vz", "sxx", "szz", "sxz", "m_vx_x", "m_vx_z", "m_vz_x", "m_vz_z",
              "m_sxx_x", "m_sxz_z", "m_sxz_x", "m_szz_z")


def el2_pad(g, vp, vs, rho):
    """-> (lam, mu, muxz, bx, bz) on the padded grid."""
    P = g.npml
    sh = (g.nz + 2 * P, g.nx + 2 * P)
    out = [np.zeros(sh) for _ in range(5)]
    lib().or_el2_pad(C.byref(g), _d(_f64(vp)), _d(_f64(vs)), _d(_f64(rho)), *[_d(o) for o in out])
    return out


def el2_step(g, model, X, src_idx=-1, mt=(0.0, 0.0, 0.0), src_val=0.0):
    model = [_f64(m) for m in model]
    X = [_f64(x) for x in X]
    Y = [np.zeros_like(X[0]) for _ in range(13)]
    mta = _f64(mt)
    lib().or_el2_step(C.byref(g), _ptrs(model), _ptrs(X), C.c_int64(src_idx), _d(mta),
                      C.c_double(src_val), _ptrs(Y))
    return Y


def el2_step_T(g, model, X, aY, src_idx=-1, mt=(0.0, 0.0, 0.0)):
    model = [_f64(m) for m in model]
    X = [_f64(x) for x in X]
    aY = [_f64(x) for x in aY]
    aX = [np.zeros_like(X[0]) for _ in range(13)]
    gM = [np.zeros_like(X[0]) for _ in range(5)]
    sb = C.c_double(0.0)
    mta = _f64(mt)
    lib().or_el2_step_T(C.byref(g), _ptrs(model), _ptrs(X), _ptrs(aY), _ptrs(aX), _ptrs(gM),
                        C.c_int64(src_idx), _d(mta), C.byref(sb))
    return aX, gM, sb.value


def el2_forward(g, vp, vs, rho, src, mt, wav, rec):
    src, rec, wav, mt = _i32(src), _i32(rec), _f64(wav), _f64(mt)
    ns, nrec = src.shape[0], rec.shape[1]
    seis = np.zeros((ns, 2, g.nt, nrec))
    if lib().or_el2_forward(C.byref(g), _d(_f64(vp)), _d(_f64(vs)), _d(_f64(rho)), C.c_int32(ns),
                            _i(src), _d(mt), _d(wav), C.c_int32(nrec), _i(rec), _d(seis)):
        raise ValueError("oracle: invalid geometry or grid")
    return seis


def el2_gradient(g, vp, vs, rho, src, mt, wav, rec, dJdd, ckpt=0):
    src, rec, wav, mt = _i32(src), _i32(rec), _f64(wav), _f64(mt)
    ns, nrec = src.shape[0], rec.shape[1]
    seis = np.zeros((ns, 2, g.nt, nrec))
    gvp, gvs, grho = np.zeros((g.nz, g.nx)), np.zeros((g.nz, g.nx)), np.zeros((g.nz, g.nx))
    if lib().or_el2_gradient(C.byref(g), _d(_f64(vp)), _d(_f64(vs)), _d(_f64(rho)), C.c_int32(ns),
                             _i(src), _d(mt), _d(wav), C.c_int32(nrec), _i(rec), _d(_f64(dJdd)),
                             C.c_int32(ckpt), _d(gvp), _d(gvs), _d(grho), _d(seis)):
        raise ValueError("oracle: invalid geometry or grid")
    return (gvp, gvs, grho), seis
