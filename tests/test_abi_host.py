"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point declared in include/molamr.h, validates arguments before
touching the device, and its BOR weights reproduce the oracle's App. D steps."""
import os
import re

import numpy as np
import pytest

from oracle import oracle as O
from paper_1806_04182_amd import molamr as M

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "molamr.h")).read()
    return sorted(set(re.findall(r"\b(mol_[a-z0-9_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    L = M.lib()
    names = _declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), n


def _hier(boxes0, N0=(8, 8, 8)):
    return M.Hierarchy(N0, (0, 0, 0), 0.125, [(1, boxes0)])


@pytest.mark.parametrize("boxes, msg", [
    ([((0, 0, 0), (7, 7, 6))], "tile the periodic domain"),
    ([((0, 0, 0), (7, 7, 7)), ((0, 0, 0), (1, 1, 1))], "overlaps"),
    ([((0, 0, 0), (8, 7, 7))], "outside"),
])
def test_create_rejects_bad_hierarchies(boxes, msg):
    with pytest.raises(M.MolError) as e:
        M.Patchset(_hier(boxes), M.System(M.MOL_WAVE))
    assert e.value.code == -1 and msg in str(e.value)


def test_create_rejects_bad_ratio():
    h = M.Hierarchy((8, 8, 8), (0, 0, 0), 0.125, [(1, [((0, 0, 0), (7, 7, 7))]), (5, [((8, 8, 8), (15, 15, 15))])])
    with pytest.raises(M.MolError) as e:
        M.Patchset(h, M.System(M.MOL_WAVE))
    assert "ratio" in str(e.value)


@pytest.mark.parametrize("R", [1, 2, 3, 4])
def test_bor_weights_match_oracle_steps(R):
    """The library's closed-form weights w_j(R, r, s) against the oracle's
    literal App. D steps applied to unit increments."""
    rng = np.random.default_rng(R)
    Un = rng.standard_normal(7)
    k = [rng.standard_normal(7) for _ in range(4)]
    for r in range(R):
        for s in range(1, 5):
            w = M.bor_weights(R, r, s)
            ref = O.bor_rk4(R, r, s, 0.37, Un, k)
            got = Un + sum(w[j] * k[j] for j in range(4))
            assert np.max(np.abs(got - ref)) < 1e-14


def test_bor_weights_table_ratio2():
    # fine step 0 of a ratio-2 step, stage 3: (3/32, 1/8, 1/16, -1/32)
    assert np.allclose(M.bor_weights(2, 0, 3), [3 / 32, 1 / 8, 1 / 16, -1 / 32], atol=1e-16)
    with pytest.raises(M.MolError):
        M.bor_weights(2, 2, 1)


@pytest.mark.parametrize("tmode,omode", [(M.MOL_TIME_BOR, O.TIME_BOR), (M.MOL_TIME_BO, O.TIME_BO),
                                         (M.MOL_TIME_BO1, O.TIME_BO1), (M.MOL_TIME_NOSUB, O.TIME_NOSUB)])
def test_time_weights_match_oracle_time_state(tmode, omode):
    """The library's weights per time-refinement strategy against the oracle's
    parent states built from the Sec. III.B definitions."""
    rng = np.random.default_rng(11 + tmode)
    Un = rng.standard_normal(9)
    k = [rng.standard_normal(9) for _ in range(4)]
    for R in ([1] if tmode == M.MOL_TIME_NOSUB else [1, 2, 3, 4]):
        for r in range(R):
            for s in range(1, 5):
                w = M.time_weights(tmode, R, r, s)
                ref = O.time_state(omode, R, r, s, 0.21, Un, k)
                got = Un + sum(w[j] * k[j] for j in range(4))
                assert np.max(np.abs(got - ref)) < 1e-14, (R, r, s)


def test_time_weights_rejects_bad_arguments():
    with pytest.raises(M.MolError):
        M.time_weights(M.MOL_TIME_NOSUB, 2, 0, 1)
    with pytest.raises(M.MolError):
        M.time_weights(7, 2, 0, 1)
    with pytest.raises(M.MolError):
        M.time_weights(M.MOL_TIME_BO, 2, 0, 5)


@pytest.mark.parametrize("tmode,omode", [(M.MOL_TIME_BOR, O.TIME_BOR), (M.MOL_TIME_BO, O.TIME_BO),
                                         (M.MOL_TIME_BO1, O.TIME_BO1), (M.MOL_TIME_NOSUB, O.TIME_NOSUB)])
def test_ssp3_time_weights_match_oracle_time_state(tmode, omode):
    """SSP-RK3 (App. C dense output, App. D BOR) weights against the oracle's
    parent states."""
    rng = np.random.default_rng(21 + tmode)
    Un = rng.standard_normal(9)
    k = [rng.standard_normal(9) for _ in range(3)]
    for R in ([1] if tmode == M.MOL_TIME_NOSUB else [1, 2, 3, 4]):
        for r in range(R):
            for s in range(1, 4):
                w = M.time_weights(tmode | M.MOL_ADV_SSPRK3, R, r, s)
                assert w[3] == 0.0
                ref = O.time_state(omode, R, r, s, 0.21, Un, k, scheme=O.SSPRK3)
                got = Un + sum(w[j] * k[j] for j in range(3))
                assert np.max(np.abs(got - ref)) < 1e-14, (R, r, s)
    with pytest.raises(M.MolError):
        M.time_weights(tmode | M.MOL_ADV_SSPRK3, 1, 0, 4)


# host clustering of refinement tags (mol_cluster) against the oracle's
@pytest.mark.parametrize("seed", [4, 5, 6, 7])
@pytest.mark.parametrize("buffer", [0, 1, 3])
def test_library_cluster_matches_oracle(seed, buffer):
    rng = np.random.default_rng(seed)
    f = (rng.random((6, 11, 13)) < 0.02).astype(np.uint8)
    assert M.cluster(f, buffer) == O.cluster(f, buffer)
    line = np.zeros((1, 1, 64), np.uint8)
    line[0, 0, [0, 5, 30, 63]] = 1
    assert M.cluster(line, buffer) == O.cluster(line, buffer)


def test_library_cluster_rejects_too_many_boxes():
    f = np.zeros((1, 1, 40), np.uint8)
    f[0, 0, ::4] = 1
    with pytest.raises(M.MolError):
        M.cluster(f, 0, max_boxes=3)


def test_set_tiling_rejects_bad_launch_shapes():
    """mol_set_tiling validates before touching the device (null patchset and
    bad shapes are argument errors)."""
    import ctypes
    t = M._Tiling((ctypes.c_int * 3)(64, 8, 4), 0, 0.0)
    assert M.lib().mol_set_tiling(None, 0, ctypes.byref(t)) == -1  # MOL_EINVAL


def test_adjoint_steps_reject_null_patchset():
    """Both reverse RK4 entry points validate their handle on the host."""
    import ctypes
    L = M.lib()
    w = (ctypes.c_void_p * 6)()
    st = (ctypes.c_void_p * 4)()
    assert L.mol_rk4_adjoint_step(None, 0, 0.1, None, None, w, None, None) == -1  # MOL_EINVAL
    assert L.mol_rk4_adjoint_step_stages(None, 0, 0.1, st, None, w, None, None) == -1
    assert "null patchset" in M.lib().mol_last_error().decode()


def test_register_staged_ccz4_loads_still_compile(tmp_path):
    """The CCZ4 stage kernel's alternative load path (halo loads staged
    through registers, -DMOL_CCZ4_DMA=0; the default path uses LDS-DMA loads)
    cross-compiles for the GPU without warnings, so the comparison build
    stays available."""
    import subprocess
    from paper_1806_04182_amd import build as B
    src = os.path.join(B.CSRC, "k_ccz4.hip")
    cmd = [B.HIPCC, *B.FLAGS, "-DMOL_CCZ4_DMA=0", "--cuda-device-only", "-x", "hip", "-c", src,
           "-o", str(tmp_path / "k_ccz4_staged.o")]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    warnings = [l for l in r.stderr.splitlines() if "warning:" in l and "packed-fp32-ops" not in l]
    assert not warnings, warnings
