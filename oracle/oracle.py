"""ctypes front of the CPU oracle (liboracle.so).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
CPU-baseline leg of the benchmark, never by the product package.

Arrays are numpy float64 patch arrays of shape (nf, nz+6, ny+6, nx+6).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

WAVE, MHD, CCZ4, MHD_GLM = 0, 1, 2, 3
RK4, SSPRK3 = 0, 1
NFIELDS = {WAVE: 2, MHD: 8, CCZ4: 25, MHD_GLM: 9}


class Params(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in (
        "sigma", "gamma_ad", "weno_eps", "weno_q", "kappa_z", "kappa_c",
        "bm_f0", "bm_f1", "gd_g", "gd_eta", "upwind", "mhd_recon", "mhd_riemann", "mhd_ch", "mhd_kpsi")]


# MHD variants: reconstruction (App. A/B) and interface flux (Sec. II.B.2)
RECON_WENO5Z, RECON_WENO5JS, RECON_WENO3 = 0, 1, 2
FLUX_LLF, FLUX_HLL, FLUX_SPLIT = 0, 1, 2


# time refinement of the sub-cycled step (Sec. III.B)
TIME_BOR, TIME_BO, TIME_BO1, TIME_NOSUB = 0, 1, 2, 3


def params(**kw) -> Params:
    d = dict(sigma=0.1, gamma_ad=5.0 / 3.0, weno_eps=-1.0, weno_q=2.0,
             kappa_z=0.1, kappa_c=0.1, bm_f0=0.0, bm_f1=2.0, gd_g=0.75,
             gd_eta=2.0, upwind=1.0, mhd_recon=0.0, mhd_riemann=0.0, mhd_ch=1.0, mhd_kpsi=0.0)
    d.update(kw)
    return Params(**d)


def build(force: bool = False) -> str:
    """Compile liboracle.so with the oracle's Makefile (gcc)."""
    if force or not os.path.exists(_LIB_PATH):
        subprocess.run(["make", "-B" if force else "-s", "-C", _HERE, "liboracle.so"],
                       check=True, capture_output=True)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        i = ctypes.c_int
        d = ctypes.c_double
        lng = ctypes.c_long
        P = ctypes.POINTER(Params)
        vp = ctypes.c_void_p
        for name in ("orc_d1", "orc_d2"):
            getattr(L, name).argtypes = [dp, lng, d]
            getattr(L, name).restype = d
        L.orc_adv.argtypes = [dp, lng, d, d]
        L.orc_adv.restype = d
        L.orc_ko.argtypes = [dp, lng, d, d]
        L.orc_ko.restype = d
        L.orc_dmix.argtypes = [dp, lng, d, lng, d]
        L.orc_dmix.restype = d
        L.orc_fill_periodic.argtypes = [dp, i, i, i, i]
        L.orc_rhs.argtypes = [i, dp, dp, i, i, i, dp, P]
        for name in ("orc_weno5z_left", "orc_weno5z_right"):
            getattr(L, name).argtypes = [dp, d, d]
            getattr(L, name).restype = d
        for name in ("orc_weno5js_left", "orc_weno5js_right", "orc_weno3_left", "orc_weno3_right"):
            getattr(L, name).argtypes = [dp, d]
            getattr(L, name).restype = d
        L.orc_mhd_interface_flux.argtypes = [dp, dp, i, d, i, dp]
        L.orc_mhd_fast_speed.argtypes = [dp, i, d]
        L.orc_mhd_fast_speed.restype = d
        L.orc_rk_run.argtypes = [i, i, dp, i, i, i, dp, d, i, P]
        L.orc_rk_scalar.argtypes = [i, d, d, dp, dp]
        L.orc_dense_rk4.argtypes = [i, i, d]
        L.orc_dense_rk4.restype = d
        L.orc_bor_rk4.argtypes = [i, i, i, d, dp, ctypes.POINTER(dp), dp, lng]
        L.orc_lagrange6.argtypes = [d, dp]
        L.orc_hier_create.argtypes = [i, i, ctypes.POINTER(i), ctypes.POINTER(i), dp, d,
                                      ctypes.POINTER(i), ctypes.POINTER(i)]
        L.orc_hier_create.restype = vp
        L.orc_hier_destroy.argtypes = [vp]
        L.orc_hier_set.argtypes = [vp, i, i, dp]
        L.orc_hier_get.argtypes = [vp, i, i, dp]
        L.orc_hier_fill_same.argtypes = [vp, i]
        L.orc_hier_step.argtypes = [vp, d, P]
        L.orc_hier_set_time_mode.argtypes = [vp, i]
        L.orc_hier_set_scheme.argtypes = [vp, i]
        L.orc_hier_set_open.argtypes = [vp, dp, dp]
        L.orc_time_state_ssp3.argtypes = [i, i, i, i, d, dp, ctypes.POINTER(dp), dp, lng]
        L.orc_dense_ssp3.argtypes = [i, i, d]
        L.orc_dense_ssp3.restype = d
        L.orc_time_state.argtypes = [i, i, i, i, d, dp, ctypes.POINTER(dp), dp, lng]
        L.orc_hier_set_parent_data.argtypes = [vp, i, i, dp, dp, dp, dp, dp]
        L.orc_hier_prolong.argtypes = [vp, i, i, i, d]
        L.orc_hier_restrict.argtypes = [vp, i]
        L.orc_hier_regrid.argtypes = [vp, vp]
        L.orc_wave_rhs_adjoint.argtypes = [dp, dp, i, i, i, dp, P]
        L.orc_fill_periodic_adjoint.argtypes = [dp, i, i, i, i]
        L.orc_wave_adjoint_run.argtypes = [dp, i, i, i, dp, dp, d, i, d, P]
        L.orc_sphere_integral.argtypes = [dp, i, i, i, i, dp, dp, d, d]
        L.orc_sphere_integral.restype = d
        L.orc_ccz4_rhs_jvp.argtypes = [dp, dp, dp, dp, i, i, i, dp, P]
        L.orc_ccz4_monitor.argtypes = [dp, dp, i, i, i, dp, P]
        L.orc_ko_monitor.argtypes = [i, dp, dp, i, i, i, dp, P]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _h3(h):
    h = np.broadcast_to(np.asarray(h, dtype=np.float64), (3,)).copy()
    return h


def dims(U: np.ndarray):
    nf, NZ, NY, NX = U.shape
    return nf, NX - 6, NY - 6, NZ - 6


def fill_periodic(U: np.ndarray) -> None:
    nf, nx, ny, nz = dims(U)
    lib().orc_fill_periodic(_p(U), nf, nx, ny, nz)


def rhs(system: int, U: np.ndarray, h, prm: Params | None = None) -> np.ndarray:
    prm = prm or params()
    nf, nx, ny, nz = dims(U)
    R = np.zeros_like(U)
    hh = _h3(h)
    lib().orc_rhs(system, _p(U), _p(R), nx, ny, nz, _p(hh), ctypes.byref(prm))
    return R


MONITORS = ("theta", "z", "hz", "lndet", "tra", "ko")


def monitor(system: int, U: np.ndarray, h, prm: Params | None = None) -> dict:
    """Constraint and dissipation monitors at every interior point (arrays of
    the interior shape): CCZ4 (Sec. V) Theta, |Z| = sqrt(gamma_ij Z^i Z^j),
    H_Z (the bracket of the Theta equation), ln det gt, tr At; every system:
    ko = sqrt(sum_f (Q_d U_f)^2), the magnitude of the dissipation term."""
    prm = prm or params()
    nf, nx, ny, nz = dims(U)
    hh = _h3(h)
    I = (slice(3, -3), slice(3, -3), slice(3, -3))
    out = {}
    if system == CCZ4:
        Mc = np.zeros((5,) + U.shape[1:])
        lib().orc_ccz4_monitor(_p(U), _p(Mc), nx, ny, nz, _p(hh), ctypes.byref(prm))
        out["theta"] = Mc[0][I].copy()
        out["z"] = np.sqrt(Mc[1][I])
        out["hz"] = Mc[2][I].copy()
        out["lndet"] = Mc[3][I].copy()
        out["tra"] = Mc[4][I].copy()
    Mk = np.zeros(U.shape[1:])
    lib().orc_ko_monitor(system, _p(U), _p(Mk), nx, ny, nz, _p(hh), ctypes.byref(prm))
    out["ko"] = np.sqrt(Mk[I])
    return out


def monitor_norms(system: int, U: np.ndarray, h, prm: Params | None = None) -> dict:
    """Per monitor: (sum |v| dV, sum v^2 dV, max |v|) over the interior
    points where v is finite, and the number of non-finite values of U at
    interior points ("nonfinite")."""
    hh = _h3(h)
    dV = hh[0] * hh[1] * hh[2]
    res = {}
    for k, v in monitor(system, U, h, prm).items():
        v = v[np.isfinite(v)]
        res[k] = (float(np.sum(np.abs(v)) * dV), float(np.sum(v * v) * dV),
                  float(np.max(np.abs(v))) if v.size else 0.0)
    res["nonfinite"] = int(np.sum(~np.isfinite(U[:, 3:-3, 3:-3, 3:-3])))
    return res


def rk_run(system: int, scheme: int, U: np.ndarray, h, dt: float, nsteps: int,
           prm: Params | None = None) -> None:
    prm = prm or params()
    nf, nx, ny, nz = dims(U)
    hh = _h3(h)
    lib().orc_rk_run(system, scheme, _p(U), nx, ny, nz, _p(hh), dt, nsteps, ctypes.byref(prm))


def rk_scalar(scheme: int, z: complex) -> complex:
    a = ctypes.c_double()
    b = ctypes.c_double()
    lib().orc_rk_scalar(scheme, z.real, z.imag, ctypes.byref(a), ctypes.byref(b))
    return complex(a.value, b.value)


def stencil(name: str, u: np.ndarray, center: int, stride: int, h: float, *extra) -> float:
    u = np.ascontiguousarray(u, dtype=np.float64)
    ptr = ctypes.cast(u.ctypes.data + 8 * center, ctypes.POINTER(ctypes.c_double))
    return getattr(lib(), "orc_" + name)(ptr, stride, h, *extra)


def dmix(u: np.ndarray, center: int, sa: int, ha: float, sb: int, hb: float) -> float:
    u = np.ascontiguousarray(u, dtype=np.float64)
    ptr = ctypes.cast(u.ctypes.data + 8 * center, ctypes.POINTER(ctypes.c_double))
    return lib().orc_dmix(ptr, sa, ha, sb, hb)


def weno(kind: str, u5: np.ndarray, eps: float, q: float = 2.0) -> float:
    u = np.ascontiguousarray(u5, dtype=np.float64)
    ptr = ctypes.cast(u.ctypes.data + 16, ctypes.POINTER(ctypes.c_double))
    if kind == "zL":
        return lib().orc_weno5z_left(ptr, eps, q)
    if kind == "zR":
        return lib().orc_weno5z_right(ptr, eps, q)
    if kind == "jsR":
        return lib().orc_weno5js_right(ptr, eps)
    if kind == "3L":
        return lib().orc_weno3_left(ptr, eps)
    if kind == "3R":
        return lib().orc_weno3_right(ptr, eps)
    return lib().orc_weno5js_left(ptr, eps)


def mhd_fast_speed(U, d: int, gam: float) -> float:
    U = np.ascontiguousarray(U, dtype=np.float64)
    return lib().orc_mhd_fast_speed(_p(U), d, gam)


def mhd_interface_flux(UL, UR, d: int, gam: float, riemann: int) -> np.ndarray:
    """Interface flux between reconstructed states (8 conserved fields)."""
    UL = np.ascontiguousarray(UL, dtype=np.float64)
    UR = np.ascontiguousarray(UR, dtype=np.float64)
    F = np.zeros(8)
    lib().orc_mhd_interface_flux(_p(UL), _p(UR), d, gam, riemann, _p(F))
    return F


def dense_rk4(j: int, m: int, theta: float) -> float:
    return lib().orc_dense_rk4(j, m, theta)


def bor_rk4(R: int, r: int, s: int, dt: float, Un: np.ndarray, k) -> np.ndarray:
    Un = np.ascontiguousarray(Un, dtype=np.float64)
    ks = [np.ascontiguousarray(x, dtype=np.float64) for x in k]
    arr = (ctypes.POINTER(ctypes.c_double) * 4)(*[_p(x) for x in ks])
    out = np.empty_like(Un)
    lib().orc_bor_rk4(R, r, s, dt, _p(Un), arr, _p(out), Un.size)
    return out


def lagrange6(xi: float) -> np.ndarray:
    w = np.zeros(6)
    lib().orc_lagrange6(xi, _p(w))
    return w


def wave_rhs_adjoint(lam: np.ndarray, h, prm: Params | None = None) -> np.ndarray:
    prm = prm or params()
    nf, nx, ny, nz = dims(lam)
    out = np.zeros_like(lam)
    lib().orc_wave_rhs_adjoint(_p(np.ascontiguousarray(lam)), _p(out), nx, ny, nz,
                               _p(_h3(h)), ctypes.byref(prm))
    return out


def fill_periodic_adjoint(A: np.ndarray) -> None:
    nf, nx, ny, nz = dims(A)
    lib().orc_fill_periodic_adjoint(_p(A), nf, nx, ny, nz)


def wave_adjoint_run(n, h, xlo, dt, nsteps, rad, prm: Params | None = None) -> np.ndarray:
    prm = prm or params()
    nx, ny, nz = n
    lam = np.zeros((2, nz + 6, ny + 6, nx + 6))
    lib().orc_wave_adjoint_run(_p(lam), nx, ny, nz, _p(_h3(h)),
                               _p(np.asarray(xlo, dtype=np.float64).copy()), dt, nsteps, rad,
                               ctypes.byref(prm))
    return lam


def sphere_integral(U: np.ndarray, field: int, xlo, h, rad: float, shift: float = 0.0) -> float:
    nf, nx, ny, nz = dims(U)
    return lib().orc_sphere_integral(_p(U), field, nx, ny, nz,
                                     _p(np.asarray(xlo, dtype=np.float64).copy()),
                                     _p(_h3(h)), rad, shift)


class Hierarchy:
    """Oracle AMR hierarchy: levels of boxes (inclusive lo/hi, level index space)."""

    def __init__(self, system: int, N0, xlo, dx0: float, levels):
        """levels: list of (ratio, [(lo3, hi3), ...]); ratio of level 0 ignored."""
        L = lib()
        self.system = system
        self.nf = NFIELDS[system]
        self.levels = levels
        ratio = (ctypes.c_int * len(levels))(*[lv[0] for lv in levels])
        npatch = (ctypes.c_int * len(levels))(*[len(lv[1]) for lv in levels])
        flat = []
        for _, boxes in levels:
            for lo, hi in boxes:
                flat += list(lo) + list(hi)
        barr = (ctypes.c_int * len(flat))(*flat)
        n0 = (ctypes.c_int * 3)(*N0)
        xl = np.asarray(xlo, dtype=np.float64).copy()
        self._h = L.orc_hier_create(system, len(levels), ratio, n0, _p(xl), dx0, npatch, barr)

    def __del__(self):
        if getattr(self, "_h", None):
            lib().orc_hier_destroy(self._h)
            self._h = None

    def shape(self, l: int, p: int):
        lo, hi = self.levels[l][1][p]
        return (self.nf, hi[2] - lo[2] + 7, hi[1] - lo[1] + 7, hi[0] - lo[0] + 7)

    def set(self, l: int, p: int, U: np.ndarray) -> None:
        U = np.ascontiguousarray(U, dtype=np.float64)
        assert U.shape == self.shape(l, p)
        lib().orc_hier_set(self._h, l, p, _p(U))

    def get(self, l: int, p: int) -> np.ndarray:
        out = np.empty(self.shape(l, p))
        lib().orc_hier_get(self._h, l, p, _p(out))
        return out

    def fill_same(self, l: int) -> None:
        lib().orc_hier_fill_same(self._h, l)

    def step(self, dt0: float, prm: Params | None = None) -> None:
        prm = prm or params()
        lib().orc_hier_step(self._h, dt0, ctypes.byref(prm))

    def set_time_mode(self, mode: int) -> None:
        lib().orc_hier_set_time_mode(self._h, mode)

    def set_open(self, v, uinf) -> None:
        """Radiative outer boundary (level 0 a single patch); v and U_inf per field."""
        self._rad = (np.ascontiguousarray(v, dtype=np.float64), np.ascontiguousarray(uinf, dtype=np.float64))
        lib().orc_hier_set_open(self._h, _p(self._rad[0]), _p(self._rad[1]))

    def set_scheme(self, scheme: int) -> None:
        """RK4 (default) or SSPRK3 for the sub-cycled step."""
        lib().orc_hier_set_scheme(self._h, scheme)

    def set_parent_data(self, l: int, p: int, Un, k) -> None:
        arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in [Un] + list(k)]
        lib().orc_hier_set_parent_data(self._h, l, p, *[_p(a) for a in arrs])

    def prolong(self, l: int, r: int, s: int, dt_parent: float) -> None:
        lib().orc_hier_prolong(self._h, l, r, s, dt_parent)

    def restrict(self, l: int) -> None:
        lib().orc_hier_restrict(self._h, l)

    def regrid_from(self, old: "Hierarchy") -> None:
        """Take the state of `old` (same level 0, other fine boxes): copies
        where old fine patches hold the point, Lagrange interpolation from the
        new parent level elsewhere (orc_hier_regrid)."""
        lib().orc_hier_regrid(self._h, old._h)


def tag(u: np.ndarray, threshold: float) -> np.ndarray:
    """Refinement criterion of the AMR wave test (Sec. IV.A): flag the points
    where |phi| >= threshold (u: the level's interior values, any shape)."""
    return (np.abs(u) >= threshold).astype(np.uint8)


def cluster(flags: np.ndarray, buffer: int) -> list:
    """Boxes covering the flagged points of a periodic (z, y, x) array: the
    flags grown by `buffer` points along each axis with wrap-around, then the
    face-connected components (no wrap: a region across a domain edge gives one
    box on each side), the bounding box ((lo x, y, z), (hi x, y, z)) of each,
    and boxes that overlap replaced by their common bounding box until none
    overlap; sorted by lower corner (z, y, x).  Sec. III.A leaves the
    clustering to SAMRAI; this is the reading used here."""
    from scipy import ndimage

    a = np.asarray(flags).astype(bool)
    for ax in range(3):
        reach = min(buffer, a.shape[ax] - 1)
        grown = a.copy()
        for o in range(1, reach + 1):
            grown |= np.roll(a, o, axis=ax) | np.roll(a, -o, axis=ax)
        a = grown
    lab, n = ndimage.label(a)  # face connectivity by default
    boxes = []
    for sl in ndimage.find_objects(lab):
        z, y, x = sl
        boxes.append([x.start, y.start, z.start, x.stop - 1, y.stop - 1, z.stop - 1])
    merged = True
    while merged:
        merged = False
        for i in range(len(boxes)):
            for j in range(i + 1, len(boxes)):
                bi, bj = boxes[i], boxes[j]
                if all(bi[3 + d] >= bj[d] and bj[3 + d] >= bi[d] for d in range(3)):
                    boxes[i] = [min(bi[d], bj[d]) for d in range(3)] + [max(bi[3 + d], bj[3 + d]) for d in range(3)]
                    del boxes[j]
                    merged = True
                    break
            if merged:
                break
    boxes.sort(key=lambda b: (b[2], b[1], b[0]))
    return [(tuple(b[:3]), tuple(b[3:])) for b in boxes]


def ccz4_rhs_jvp(U: np.ndarray, V: np.ndarray, h, prm: Params | None = None):
    """(R(U), R'(U) V) of the CCZ4 right-hand side on a ghosted patch array,
    the derivative exact up to rounding (dual-number build of the oracle)."""
    prm = prm or params()
    nf, nx, ny, nz = dims(U)
    assert nf == 25 and V.shape == U.shape
    R = np.zeros_like(U)
    RV = np.zeros_like(U)
    lib().orc_ccz4_rhs_jvp(_p(U), _p(np.ascontiguousarray(V)), _p(R), _p(RV), nx, ny, nz, _p(_h3(h)),
                           ctypes.byref(prm))
    return R, RV


def ccz4_rhs_vjp_periodic(U: np.ndarray, lam: np.ndarray, h, prm: Params | None = None) -> np.ndarray:
    """Transpose of the CCZ4 right-hand side of a periodic patch applied to lam:
    (lamU)_{f,p} = sum over interior points c of lam(c) . d R(c) / d U_f(p),
    where U's ghosts are the periodic images of its interior.  Assembled
    column by column from exact JVPs (one per interior value): small patches
    only.  U is a ghosted array with filled ghosts; lam and the result are
    interior arrays (25, nz, ny, nx)."""
    nf, nx, ny, nz = dims(U)
    out = np.zeros((nf, nz, ny, nx))
    V = np.zeros_like(U)
    for f in range(nf):
        for k in range(nz):
            for j in range(ny):
                for i in range(nx):
                    V[:] = 0.0
                    V[f, k + 3, j + 3, i + 3] = 1.0
                    fill_periodic(V)
                    _, RV = ccz4_rhs_jvp(U, V, h, prm)
                    out[f, k, j, i] = np.sum(lam * RV[:, 3:-3, 3:-3, 3:-3])
    return out


def time_state(mode: int, R: int, r: int, s: int, dt: float, Un: np.ndarray, k, scheme: int = 0) -> np.ndarray:
    """Parent state feeding fine step r, stage s for a time-refinement mode."""
    out = np.zeros_like(Un)
    arr = (ctypes.POINTER(ctypes.c_double) * 4)(*[_p(np.ascontiguousarray(kk)) for kk in k])
    fn = lib().orc_time_state_ssp3 if scheme == SSPRK3 else lib().orc_time_state
    fn(mode, R, r, s, dt, _p(Un), arr, _p(out), Un.size)
    return out


def dense_ssp3(j: int, m: int, theta: float) -> float:
    return lib().orc_dense_ssp3(j, m, theta)



def ccz4_puncture_at(x, y, z, holes) -> np.ndarray:
    """Puncture initial data of Sec. V at the points (x, y, z) (arrays of one
    shape), for holes [(m, centre(3), P(3), S(3)), ...]: the 25 CCZ4 fields.
    Conformal factor psi = 1 + sum_A m_A / (2 r_A) (eq. conformal_factor,
    Brill-Lindquist); chi = psi^-4, gt_ij = delta_ij, trKhat = Theta = 0,
    Ghat^i = beta^i = B^i = 0, alpha = psi^-2 (the paper's initial lapse);
    At_ij = psi^-6 times the sum over holes of the Bowen-York solution
      3/(2 r^2) [P_i n_j + P_j n_i - (delta_ij - n_i n_j) P^k n_k]
      + 3/r^3 [eps_kil S^l n^k n_j + eps_kjl S^l n^k n_i],
    n = (x - c)/r.  No point may coincide with a puncture."""
    x = [np.asarray(x, dtype=np.float64), np.asarray(y, dtype=np.float64), np.asarray(z, dtype=np.float64)]
    psi = np.ones_like(x[0])
    for m, c, _, _ in holes:
        r = np.sqrt((x[0] - c[0]) ** 2 + (x[1] - c[1]) ** 2 + (x[2] - c[2]) ** 2)
        psi = psi + m / (2.0 * r)
    eps = np.zeros((3, 3, 3))
    eps[0, 1, 2] = eps[1, 2, 0] = eps[2, 0, 1] = 1.0
    eps[0, 2, 1] = eps[2, 1, 0] = eps[1, 0, 2] = -1.0
    A = np.zeros((3, 3) + x[0].shape)
    for m, c, P, S in holes:
        r = np.sqrt((x[0] - c[0]) ** 2 + (x[1] - c[1]) ** 2 + (x[2] - c[2]) ** 2)
        n = [(x[d] - c[d]) / r for d in range(3)]
        Pn = P[0] * n[0] + P[1] * n[1] + P[2] * n[2]
        for i in range(3):
            for j in range(3):
                dij = 1.0 if i == j else 0.0
                mom = 1.5 / r ** 2 * (P[i] * n[j] + P[j] * n[i] - (dij - n[i] * n[j]) * Pn)
                spin = 0.0
                for k in range(3):
                    for l in range(3):
                        spin = spin + (eps[k, i, l] * n[j] + eps[k, j, l] * n[i]) * S[l] * n[k]
                A[i, j] = A[i, j] + mom + 3.0 / r ** 3 * spin
    A = A / psi ** 6
    out = np.zeros((25,) + x[0].shape)
    out[0] = psi ** -4
    for q, (i, j) in enumerate(((0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2))):
        out[1 + q] = 1.0 if i == j else 0.0
        out[8 + q] = A[i, j]
    out[18] = psi ** -2
    return out


def ccz4_puncture(n, h, lo, xlo, holes) -> np.ndarray:
    """ccz4_puncture_at on the points x_d = xlo_d + (lo_d + i) h of an
    n[0] x n[1] x n[2] block, as a (25, n[2], n[1], n[0]) array."""
    ax = [xlo[d] + (lo[d] + np.arange(n[d])) * h for d in range(3)]
    Z, Y, X = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    return ccz4_puncture_at(X, Y, Z, holes)
