"""Python binding of libmolamr (include/molamr.h).

Argument marshalling only: every operation runs in the HIP library.  Device
buffers are torch float64 tensors on the GPU (passed by pointer), streams are
torch streams.  The library must be built (``paper_1806_04182_amd.build``);
importing this module on a machine without it raises instead of falling back.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
from dataclasses import dataclass, field
from typing import Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("MOLAMR_LIB", os.path.join(HERE, "libmolamr.so"))

MOL_WAVE, MOL_MHD, MOL_CCZ4, MOL_MHD_GLM = 0, 1, 2, 3
MOL_RK4, MOL_SSPRK3 = 0, 1
MOL_BATCHED, MOL_PLAIN = 0, 1
MOL_RECON_WENO5Z, MOL_RECON_WENO5JS, MOL_RECON_WENO3 = 0, 1, 2
MOL_FLUX_LLF, MOL_FLUX_HLL, MOL_FLUX_SPLIT = 0, 1, 2
# time-refinement strategies (Sec. III.B), or-ed into the mode of advance()
MOL_TIME_BOR, MOL_TIME_BO, MOL_TIME_BO1, MOL_TIME_NOSUB = 0, 16, 32, 48
MOL_ADV_SSPRK3 = 64  # SSP-RK3 steps in advance() (or-ed into the mode)
MOL_ADJOINT_SCRATCH_BYTES = 64 << 20  # static workspace of mol_rhs_adjoint_noalloc
MOL_MON_THETA, MOL_MON_Z, MOL_MON_HZ, MOL_MON_LNDET, MOL_MON_TRA, MOL_MON_KO = (1 << q for q in range(6))
MOL_MON_ALL, MOL_MON_COUNT = 0x3F, 6
MOL_MON_OUT = 3 * MOL_MON_COUNT + 1
MONITORS = ("theta", "z", "hz", "lndet", "tra", "ko")
GHOST = 3
NFIELDS = {MOL_WAVE: 2, MOL_MHD: 8, MOL_CCZ4: 25, MOL_MHD_GLM: 9}


class MolError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"molamr error {code}: {msg}")
        self.code = code


class _Hier(ctypes.Structure):
    _fields_ = [("nlevels", ctypes.c_int), ("N0", ctypes.c_int * 3), ("xlo", ctypes.c_double * 3),
                ("dx0", ctypes.c_double), ("ratio", ctypes.POINTER(ctypes.c_int)),
                ("npatch", ctypes.POINTER(ctypes.c_int)), ("boxes", ctypes.POINTER(ctypes.c_int)),
                ("open", ctypes.c_int)]


class _Sys(ctypes.Structure):
    _fields_ = [("system", ctypes.c_int), ("upwind", ctypes.c_int)] + [
        (n, ctypes.c_double) for n in ("sigma", "gamma_ad", "weno_eps", "weno_q", "kappa_z", "kappa_c",
                                       "bm_f0", "bm_f1", "gd_g", "gd_eta")] + [
        ("mhd_recon", ctypes.c_int), ("mhd_flux", ctypes.c_int), ("mhd_ch", ctypes.c_double),
        ("mhd_kpsi", ctypes.c_double)]


class _Tiling(ctypes.Structure):
    _fields_ = [("tdim", ctypes.c_int * 3), ("order", ctypes.c_int), ("ms", ctypes.c_double)]


class _LevelState(ctypes.Structure):
    _fields_ = [("U", ctypes.c_void_p), ("S0", ctypes.c_void_p), ("S1", ctypes.c_void_p),
                ("acc", ctypes.c_void_p), ("k", ctypes.c_void_p * 4)]


_lib = None


def lib():
    """Load libmolamr.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_1806_04182_amd.build")
        # torch brings its own HIP runtime; the library must bind to the same
        # one, so torch is loaded first (a runtime loaded by the library first
        # would leave torch without a usable device)
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        vp, i, d = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
        i64p = ctypes.POINTER(ctypes.c_int64)
        i32p = ctypes.POINTER(ctypes.c_int32)
        dp = ctypes.POINTER(ctypes.c_double)
        sig = {
            "mol_create_patchset": ([ctypes.POINTER(_Hier), ctypes.POINTER(_Sys), ctypes.POINTER(vp)], i),
            "mol_create_patchset_from": ([ctypes.POINTER(_Hier), ctypes.POINTER(_Sys), vp, ctypes.POINTER(vp)], i),
            "mol_destroy_patchset": ([vp], None),
            "mol_last_error": ([], ctypes.c_char_p),
            "mol_nfields": ([vp], i),
            "mol_level_layout": ([vp, i, i64p, i64p, i32p, i64p, i32p], i),
            "mol_level_npatch": ([vp, i], i),
            "mol_fill_ghosts": ([vp, i, vp, i, vp], i),
            "mol_rhs": ([vp, i, vp, vp, vp], i),
            "mol_rk_stage": ([vp, i, i, i, d, vp, vp, vp, vp, vp, vp], i),
            "mol_prolong": ([vp, i, i, i, vp, ctypes.POINTER(vp), vp, vp], i),
            "mol_bor_weights": ([i, i, i, dp], i),
            "mol_time_weights": ([i, i, i, i, dp], i),
            "mol_set_radiative": ([vp, dp, dp], i),
            "mol_restrict": ([vp, i, vp, vp, vp], i),
            "mol_rhs_adjoint": ([vp, i, vp, vp, vp, vp, vp], i),
            "mol_rhs_adjoint_noalloc": ([vp, i, vp, vp, vp, vp], i),
            "mol_adjoint_workspace": ([vp, i], ctypes.c_int64),
            "mol_fill_ghosts_adjoint": ([vp, i, vp, vp], i),
            "mol_rk4_adjoint_step": ([vp, i, d, vp, vp, ctypes.POINTER(vp), vp, vp], i),
            "mol_rk4_adjoint_step_stages": ([vp, i, d, ctypes.POINTER(vp), vp, ctypes.POINTER(vp), vp, vp], i),
            "mol_norms": ([vp, i, vp, i, d, d, vp, vp], i),
            "mol_box_norms": ([vp, i, vp, i, d, dp, dp, vp, vp], i),
            "mol_sphere_adjoint": ([vp, i, i, d, d, vp, vp], i),
            "mol_monitor": ([vp, i, vp, ctypes.c_uint32, vp, vp, vp], i),
            "mol_ccz4_puncture": ([vp, i, i, dp, i, vp, vp], i),
            "mol_wave_gaussian": ([vp, i, dp, vp, vp], i),
            "mol_wave_gaussian_vjp": ([vp, i, dp, vp, vp, vp], i),
            "mol_ccz4_lapse_pulse": ([vp, i, dp, vp, vp], i),
            "mol_ccz4_lapse_pulse_vjp": ([vp, i, dp, vp, vp, vp], i),
            "mol_advance": ([vp, ctypes.POINTER(_LevelState), d, i, vp], i),
            "mol_advance_steps": ([vp, ctypes.POINTER(_LevelState), d, i, i, vp], i),
            "mol_graph_create": ([vp, ctypes.POINTER(_LevelState), d, ctypes.POINTER(vp)], i),
            "mol_graph_create_steps": ([vp, ctypes.POINTER(_LevelState), d, i, ctypes.POINTER(vp)], i),
            "mol_graph_launch": ([vp, vp], i),
            "mol_graph_destroy": ([vp], None),
            "mol_tag": ([vp, i, vp, i, d, vp, vp], i),
            "mol_autotune": ([vp, i, ctypes.POINTER(_LevelState), d, i, ctypes.POINTER(_Tiling), vp], i),
            "mol_set_tiling": ([vp, i, ctypes.POINTER(_Tiling)], i),
            "mol_cluster": ([ctypes.POINTER(ctypes.c_uint8), ctypes.POINTER(ctypes.c_int), i, i,
                             ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)], i),
            "mol_regrid_create": ([vp, vp, ctypes.POINTER(vp)], i),
            "mol_regrid_apply": ([vp, ctypes.POINTER(vp), ctypes.POINTER(vp), vp], i),
            "mol_regrid_destroy": ([vp], None),
        }
        for name, (args, res) in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def exported_symbols() -> list[str]:
    return [n for n in dir(lib()) if n.startswith("mol_")]


def _check(rc: int) -> None:
    if rc != 0:
        raise MolError(rc, lib().mol_last_error().decode())


def _ptr(t) -> int | None:
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


def _stream(stream) -> int | None:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return stream if isinstance(stream, int) else stream.cuda_stream


@dataclass
class System:
    system: int
    sigma: float = 0.1
    gamma_ad: float = 5.0 / 3.0
    weno_eps: float = -1.0
    weno_q: float = 2.0
    kappa_z: float = 0.1
    kappa_c: float = 0.1
    bm_f0: float = 0.0
    bm_f1: float = 2.0
    gd_g: float = 0.75
    gd_eta: float = 2.0
    upwind: int = 1
    mhd_recon: int = 0  # MOL_RECON_*
    mhd_flux: int = 0   # MOL_FLUX_*
    mhd_ch: float = 1.0    # MOL_MHD_GLM cleaning speed
    mhd_kpsi: float = 0.0  # MOL_MHD_GLM damping

    def _c(self) -> _Sys:
        return _Sys(self.system, int(self.upwind), self.sigma, self.gamma_ad, self.weno_eps, self.weno_q,
                    self.kappa_z, self.kappa_c, self.bm_f0, self.bm_f1, self.gd_g, self.gd_eta,
                    int(self.mhd_recon), int(self.mhd_flux), self.mhd_ch, self.mhd_kpsi)


@dataclass
class Hierarchy:
    N0: tuple
    xlo: tuple
    dx0: float
    levels: list  # [(ratio, [((lo), (hi)), ...]), ...]
    open: bool = False  # radiative outer boundary instead of a periodic level 0

    def _c(self):
        ratio = (ctypes.c_int * len(self.levels))(*[lv[0] for lv in self.levels])
        npatch = (ctypes.c_int * len(self.levels))(*[len(lv[1]) for lv in self.levels])
        flat = [v for _, boxes in self.levels for lo, hi in boxes for v in (*lo, *hi)]
        boxes = (ctypes.c_int * len(flat))(*flat)
        h = _Hier(len(self.levels), (ctypes.c_int * 3)(*self.N0), (ctypes.c_double * 3)(*self.xlo),
                  self.dx0, ratio, npatch, boxes, int(bool(self.open)))
        return h, (ratio, npatch, boxes)


class Patchset:
    """A hierarchy of patches with its device schedules (mol_create_patchset;
    with `prev`, mol_create_patchset_from: the leading levels that match
    prev's take its schedules)."""

    def __init__(self, hier: Hierarchy, system: System, prev: "Patchset | None" = None):
        h, keep = hier._c()
        s = system._c()
        out = ctypes.c_void_p()
        if prev is None:
            _check(lib().mol_create_patchset(ctypes.byref(h), ctypes.byref(s), ctypes.byref(out)))
        else:
            _check(lib().mol_create_patchset_from(ctypes.byref(h), ctypes.byref(s), prev._h, ctypes.byref(out)))
        self._h = out
        self.hier = hier
        self.system = system
        self.nf = lib().mol_nfields(self._h)
        self.nlev = len(hier.levels)
        self.layouts = [self.level_layout(l) for l in range(self.nlev)]

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.mol_destroy_patchset(self._h)
            self._h = None

    # ---- layout -------------------------------------------------------
    def level_layout(self, level: int):
        np_ = lib().mol_level_npatch(self._h, level)
        if np_ < 0:
            _check(np_)
        n = ctypes.c_int64()
        offs = (ctypes.c_int64 * np_)()
        dims = (ctypes.c_int32 * (3 * np_))()
        fss = (ctypes.c_int64 * np_)()
        pxs = (ctypes.c_int32 * np_)()
        _check(lib().mol_level_layout(self._h, level, ctypes.byref(n), offs, dims, fss, pxs))
        return dict(nelems=n.value, offsets=list(offs), dims=[tuple(dims[3 * p:3 * p + 3]) for p in range(np_)],
                    fstrides=list(fss), pitches=list(pxs))

    def _view(self, level: int, buf, p: int, nf: int):
        """(nf, nz+6, ny+6, nx+6) view of patch p inside a level buffer."""
        L = self.layouts[level]
        nx, ny, nz = L["dims"][p]
        px, fs, off = L["pitches"][p], L["fstrides"][p], L["offsets"][p]
        blk = buf[off:off + nf * fs].reshape(nf, fs)
        return blk[:, :px * (ny + 6) * (nz + 6)].reshape(nf, nz + 6, ny + 6, px)[..., :nx + 6]

    def alloc(self, level: int, device="cuda"):
        import torch
        return torch.zeros(self.layouts[level]["nelems"], dtype=torch.float64, device=device)

    def pack(self, level: int, patches: Sequence[np.ndarray]) -> np.ndarray:
        """Patch arrays (nf, nz+6, ny+6, nx+6) -> one host level buffer."""
        buf = np.zeros(self.layouts[level]["nelems"])
        for p, a in enumerate(patches):
            self._view(level, buf, p, a.shape[0])[...] = a
        return buf

    def unpack(self, level: int, buf, nf: int | None = None) -> list[np.ndarray]:
        if not isinstance(buf, np.ndarray):
            buf = buf.detach().cpu().numpy()
        nf = nf or self.nf
        return [self._view(level, buf, p, nf).copy() for p in range(len(self.layouts[level]["dims"]))]

    # ---- operations (same names as the C ABI) ---------------------------
    def fill_ghosts(self, level, U, nf=0, stream=None):
        _check(lib().mol_fill_ghosts(self._h, level, _ptr(U), nf, _stream(stream)))

    def rhs(self, level, U, dUdt, stream=None):
        _check(lib().mol_rhs(self._h, level, _ptr(U), _ptr(dUdt), _stream(stream)))

    def rk_stage(self, level, scheme, stage, dt, Un, Us, Acc, Uout, k_store=None, stream=None):
        _check(lib().mol_rk_stage(self._h, level, scheme, stage, dt, _ptr(Un), _ptr(Us), _ptr(Acc),
                                  _ptr(Uout), _ptr(k_store), _stream(stream)))

    def prolong(self, fine_level, r, stage, Un_c, k_c, U_f, stream=None):
        arr = (ctypes.c_void_p * 4)(*[_ptr(k) for k in k_c])
        _check(lib().mol_prolong(self._h, fine_level, r, stage, _ptr(Un_c), arr, _ptr(U_f), _stream(stream)))

    def restrict(self, fine_level, U_f, U_c, stream=None):
        _check(lib().mol_restrict(self._h, fine_level, _ptr(U_f), _ptr(U_c), _stream(stream)))

    def rhs_adjoint(self, level, U, lam, lamU, work=None, stream=None):
        _check(lib().mol_rhs_adjoint(self._h, level, _ptr(U), _ptr(lam), _ptr(lamU), _ptr(work), _stream(stream)))

    def rhs_adjoint_noalloc(self, level, U, lam, lamU, stream=None):
        """rhs_adjoint with the library's static workspace (allocates nothing)."""
        _check(lib().mol_rhs_adjoint_noalloc(self._h, level, _ptr(U), _ptr(lam), _ptr(lamU), _stream(stream)))

    def adjoint_workspace(self, level) -> int:
        n = lib().mol_adjoint_workspace(self._h, level)
        if n < 0:
            _check(int(n))
        return int(n)

    def alloc_work(self, level, device="cuda"):
        """Workspace for rhs_adjoint / rk4_adjoint_step (None when none is needed)."""
        import torch
        n = self.adjoint_workspace(level)
        return torch.empty(n, dtype=torch.float64, device=device) if n > 0 else None

    def fill_ghosts_adjoint(self, level, lamU, stream=None):
        _check(lib().mol_fill_ghosts_adjoint(self._h, level, _ptr(lamU), _stream(stream)))

    def rk4_adjoint_step(self, level, dt, lam, w, Un=None, work=None, stream=None):
        """w: 3 (wave) or 6 (CCZ4) level-size work buffers."""
        ws = list(w) + [None] * (6 - len(w))
        arr = (ctypes.c_void_p * 6)(*[_ptr(x) for x in ws])
        _check(lib().mol_rk4_adjoint_step(self._h, level, dt, _ptr(Un), _ptr(lam), arr, _ptr(work), _stream(stream)))

    def rk4_adjoint_step_stages(self, level, dt, lam, w, stages=None, work=None, stream=None):
        """Reverse RK4 step from kept stage states: stages = [U_1 = U^n, U_2,
        U_3, U_4] (ghosts filled; None for the wave); w: 3 level-size work
        buffers."""
        st = (ctypes.c_void_p * 4)(*[_ptr(x) for x in stages]) if stages is not None else None
        arr = (ctypes.c_void_p * 3)(*[_ptr(x) for x in w])
        _check(lib().mol_rk4_adjoint_step_stages(self._h, level, dt, st, _ptr(lam), arr, _ptr(work), _stream(stream)))

    def norms(self, level, U, field, shift, radius, out_dev, stream=None):
        _check(lib().mol_norms(self._h, level, _ptr(U), field, shift, radius, _ptr(out_dev), _stream(stream)))

    def monitor(self, level, U, which, out_dev, pointwise=None, stream=None):
        """Constraint / dissipation monitors (mol_monitor): out_dev holds
        MOL_MON_OUT doubles (L1, sum of squares and max per monitor, then
        the count of non-finite values)."""
        _check(lib().mol_monitor(self._h, level, _ptr(U), which, _ptr(pointwise), _ptr(out_dev), _stream(stream)))

    def ccz4_puncture(self, level, holes, U, whole=False, stream=None):
        """Puncture initial data (mol_ccz4_puncture); holes: [(m, centre(3),
        P(3), S(3)), ...]; whole: also the ghost points."""
        flat = [float(v) for m, c, P, S in holes for v in (m, *c, *P, *S)]
        arr = (ctypes.c_double * len(flat))(*flat)
        _check(lib().mol_ccz4_puncture(self._h, level, len(holes), arr, 1 if whole else 0, _ptr(U), _stream(stream)))

    def set_radiative(self, v, uinf):
        """Per-field speed and value at infinity of the radiative boundary."""
        nf = self.nf
        va, ua = (ctypes.c_double * nf)(*v), (ctypes.c_double * nf)(*uinf)
        _check(lib().mol_set_radiative(self._h, va, ua))

    def box_norms(self, level, U, field, shift, lo, hi, out_dev, stream=None):
        """norms() restricted to interior points with lo <= x <= hi."""
        blo, bhi = (ctypes.c_double * 3)(*lo), (ctypes.c_double * 3)(*hi)
        _check(lib().mol_box_norms(self._h, level, _ptr(U), field, shift, blo, bhi, _ptr(out_dev),
                                   _stream(stream)))

    def sphere_adjoint(self, level, field, radius, scale, lam, stream=None):
        _check(lib().mol_sphere_adjoint(self._h, level, field, radius, scale, _ptr(lam), _stream(stream)))

    def wave_gaussian(self, level, prm, U, stream=None):
        p = (ctypes.c_double * 5)(*prm)
        _check(lib().mol_wave_gaussian(self._h, level, p, _ptr(U), _stream(stream)))

    def wave_gaussian_vjp(self, level, prm, lam, grad_dev, stream=None):
        p = (ctypes.c_double * 5)(*prm)
        _check(lib().mol_wave_gaussian_vjp(self._h, level, p, _ptr(lam), _ptr(grad_dev), _stream(stream)))

    def ccz4_lapse_pulse(self, level, prm, U, stream=None):
        p = (ctypes.c_double * 5)(*prm)
        _check(lib().mol_ccz4_lapse_pulse(self._h, level, p, _ptr(U), _stream(stream)))

    def ccz4_lapse_pulse_vjp(self, level, prm, lam, grad_dev, stream=None):
        p = (ctypes.c_double * 5)(*prm)
        _check(lib().mol_ccz4_lapse_pulse_vjp(self._h, level, p, _ptr(lam), _ptr(grad_dev), _stream(stream)))

    def _states(self, states):
        arr = (_LevelState * self.nlev)()
        for l, st in enumerate(states):
            arr[l].U = _ptr(st["U"])
            arr[l].S0 = _ptr(st["S0"])
            arr[l].S1 = _ptr(st["S1"])
            arr[l].acc = _ptr(st["acc"])
            ks = st.get("k") or [None] * 4
            for j in range(4):
                arr[l].k[j] = _ptr(ks[j])
        return arr

    def advance(self, states, dt0, mode=MOL_BATCHED, stream=None):
        """One level-0 step; mode = MOL_BATCHED or MOL_PLAIN | MOL_TIME_*."""
        _check(lib().mol_advance(self._h, self._states(states), dt0, mode, _stream(stream)))

    def advance_steps(self, states, dt0, nsteps, mode=MOL_BATCHED, stream=None):
        """nsteps level-0 steps in one call (mol_advance_steps)."""
        _check(lib().mol_advance_steps(self._h, self._states(states), dt0, nsteps, mode, _stream(stream)))

    def graph_create(self, states, dt0, nsteps=1):
        """A HIP graph of nsteps level-0 steps (mol_graph_create_steps)."""
        g = ctypes.c_void_p()
        _check(lib().mol_graph_create_steps(self._h, self._states(states), dt0, nsteps, ctypes.byref(g)))
        return Graph(g)

    def period(self, level: int) -> tuple:
        """Index extent of a level: N0 times the ratios up to it."""
        f = 1
        for l in range(1, level + 1):
            f *= self.hier.levels[l][0]
        return tuple(n * f for n in self.hier.N0)

    def tag(self, level, U, field, threshold, flags_dev, stream=None):
        """Set flags_dev (uint8, index extent of the level, x fastest) to 1
        where |U[field]| >= threshold on the level's interior points."""
        _check(lib().mol_tag(self._h, level, _ptr(U), field, threshold, _ptr(flags_dev), _stream(stream)))

    def autotune(self, level, state, dt, reps=5, stream=None) -> dict:
        """Time the level's stage launch shapes and patch orders and keep the
        fastest (mol_autotune); state: the level's dict from alloc_states
        (U read, S0/S1/acc overwritten)."""
        arr = self._states([state])  # the entry point reads the first record
        t = _Tiling()
        _check(lib().mol_autotune(self._h, level, arr, dt, reps, ctypes.byref(t), _stream(stream)))
        return {"tdim": tuple(t.tdim), "order": t.order, "ms": t.ms}

    def set_tiling(self, level, tdim, order=0):
        t = _Tiling((ctypes.c_int * 3)(*tdim), order, 0.0)
        _check(lib().mol_set_tiling(self._h, level, ctypes.byref(t)))

    def tiling_key(self, level) -> str:
        """Key of a level's stage launches in an autotuning cache: the device,
        the library build (hash of the shared object), the system and the
        level's ratio and boxes (in order: the tile orders depend on it)."""
        import hashlib
        import json
        import torch
        desc = {"device": torch.cuda.get_device_name(), "system": dataclasses.asdict(self.system),
                "ratio": self.hier.levels[level][0], "boxes": [[list(lo), list(hi)] for lo, hi in
                                                               self.hier.levels[level][1]],
                "lib": _lib_digest()}
        return hashlib.sha256(json.dumps(desc, sort_keys=True).encode()).hexdigest()

    def autotune_cached(self, level, state, dt, cache, reps=5, stream=None) -> dict:
        """autotune with a JSON cache file: a level seen before (same key)
        takes its recorded tiling without timing anything; otherwise the
        level is tuned and the result recorded.  Returns the tiling and
        whether it came from the cache."""
        import json
        key = self.tiling_key(level)
        try:
            with open(cache) as fh:
                table = json.load(fh)
        except (OSError, ValueError):
            table = {}
        if key in table:
            rec = table[key]
            self.set_tiling(level, rec["tdim"], rec["order"])
            return {"tdim": tuple(rec["tdim"]), "order": rec["order"], "ms": rec["ms"], "cached": True}
        res = self.autotune(level, state, dt, reps, stream)
        table[key] = {"tdim": list(res["tdim"]), "order": res["order"], "ms": res["ms"]}
        tmp = f"{cache}.{os.getpid()}.tmp"
        with open(tmp, "w") as fh:
            json.dump(table, fh, indent=1, sort_keys=True)
        os.replace(tmp, cache)
        return dict(res, cached=False)

    def alloc_states(self, device="cuda"):
        """Device buffers for mol_advance: U, S0, S1, acc and (when a finer
        level exists) k[4] per level."""
        out = []
        for l in range(self.nlev):
            st = {n: self.alloc(l, device) for n in ("U", "S0", "S1", "acc")}
            st["k"] = [self.alloc(l, device) for _ in range(4)] if l + 1 < self.nlev else None
            out.append(st)
        return out


_LIB_DIGEST = None


def _lib_digest() -> str:
    """sha256 of the loaded library file (an autotuning cache entry holds only
    for the build that measured it)."""
    global _LIB_DIGEST
    if _LIB_DIGEST is None:
        import hashlib
        with open(LIB_PATH, "rb") as fh:
            _LIB_DIGEST = hashlib.sha256(fh.read()).hexdigest()
    return _LIB_DIGEST


def cluster(flags: np.ndarray, buffer: int, max_boxes: int = 4096) -> list:
    """Boxes ((lo), (hi)) covering the tagged points of a (z, y, x) uint8 array
    after a periodic dilation by `buffer` points (mol_cluster)."""
    f = np.ascontiguousarray(flags, dtype=np.uint8)
    dims = (ctypes.c_int * 3)(f.shape[2], f.shape[1], f.shape[0])
    out = (ctypes.c_int * (6 * max_boxes))()
    nb = ctypes.c_int()
    _check(lib().mol_cluster(f.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), dims, int(buffer), max_boxes, out,
                             ctypes.byref(nb)))
    return [(tuple(out[6 * q:6 * q + 3]), tuple(out[6 * q + 3:6 * q + 6])) for q in range(nb.value)]


class Regrid:
    """Transfer plan from an old patchset to a new one (mol_regrid_create)."""

    def __init__(self, ps_new: "Patchset", ps_old: "Patchset"):
        g = ctypes.c_void_p()
        _check(lib().mol_regrid_create(ps_new._h, ps_old._h, ctypes.byref(g)))
        self._r = g
        self._keep = (ps_new, ps_old)
        self.nlev = ps_new.nlev

    def apply(self, U_old, U_new, stream=None):
        a = (ctypes.c_void_p * self.nlev)(*[_ptr(x) for x in U_old])
        b = (ctypes.c_void_p * self.nlev)(*[_ptr(x) for x in U_new])
        _check(lib().mol_regrid_apply(self._r, a, b, _stream(stream)))

    def __del__(self):
        if getattr(self, "_r", None) and _lib is not None:
            _lib.mol_regrid_destroy(self._r)
            self._r = None


class Graph:
    def __init__(self, handle):
        self._g = handle

    def launch(self, stream=None):
        _check(lib().mol_graph_launch(self._g, _stream(stream)))

    def __del__(self):
        if getattr(self, "_g", None) and _lib is not None:
            _lib.mol_graph_destroy(self._g)
            self._g = None


def bor_weights(R: int, r: int, stage: int) -> np.ndarray:
    w = (ctypes.c_double * 4)()
    _check(lib().mol_bor_weights(R, r, stage, w))
    return np.array(list(w))


def time_weights(tmode: int, R: int, r: int, stage: int) -> np.ndarray:
    """Weights w_1..w_4 of the prolonged parent state U^n + sum_j w_j k_j
    for fine step r, stage `stage`, under strategy `tmode` (MOL_TIME_*)."""
    w = (ctypes.c_double * 4)()
    _check(lib().mol_time_weights(tmode, R, r, stage, w))
    return np.array(list(w))


def single_patch(n, xlo, dx) -> Hierarchy:
    """One periodic patch covering an n[0] x n[1] x n[2] domain."""
    return Hierarchy(tuple(n), tuple(xlo), dx, [(1, [((0, 0, 0), tuple(x - 1 for x in n))])])
