"""Checkpoint and restart: the file round trip on the host, and on the GPU
the identity n steps = n/2 steps + checkpoint + restore into a new patchset
+ n/2 steps, bit for bit over every packed level buffer (ghosts included),
for the wave and CCZ4 on the three-level ragged hierarchy and the Brio-Wu
tube with FMR under SSP-RK3 and BOR."""
import types

import numpy as np
import pytest

from paper_1806_04182_amd import checkpoint as C
from paper_1806_04182_amd import molamr as M


def _fake_ps(hier, system, sizes):
    return types.SimpleNamespace(hier=hier, system=system, nlev=len(sizes),
                                 layouts=[{"nelems": n} for n in sizes])


def test_file_round_trip_on_the_host(tmp_path):
    import torch
    levels = [(1, [((0, 0, 0), (7, 7, 7))]), (2, [((4, 4, 4), (9, 11, 9)), ((10, 4, 4), (11, 11, 9))])]
    hier = M.Hierarchy((8, 8, 8), (-1.0, -0.5, 0.25), 0.25, levels, open=True)
    system = M.System(M.MOL_MHD, sigma=0.0, gamma_ad=2.0, mhd_recon=M.MOL_RECON_WENO3, mhd_flux=M.MOL_FLUX_HLL)
    rng = np.random.default_rng(0)
    Us = [torch.from_numpy(rng.standard_normal(n)) for n in (1000, 2345)]
    Us[1][7] = float("nan")
    ps = _fake_ps(hier, system, [1000, 2345])
    p = tmp_path / "ck.safetensors"
    C.save(p, ps, Us, t=0.1 + 0.2, step=17, extra={"tmode": 3})
    h2, s2, U2, t, step, extra = C.read(p)
    assert h2 == hier and s2 == system
    assert t == 0.1 + 0.2 and step == 17 and extra == {"tmode": 3}
    for a, b in zip(Us, U2):
        assert np.array_equal(a.numpy().view(np.uint64), b.numpy().view(np.uint64))
    with pytest.raises(ValueError, match="level states"):
        C.save(p, ps, Us[:1])
    with pytest.raises(ValueError, match="float64"):
        C.save(p, ps, [Us[0], Us[1][:-1]])


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU test needs a GPU"
    return torch


def _packed(ps, st):
    return [s["U"].cpu().numpy().copy() for s in st]


def _identity(tmp_path, ps, st, nsteps, step_fn):
    """Run nsteps; separately run nsteps/2, checkpoint, restore, run the rest."""
    torch = _torch()
    start = _packed(ps, st)
    for _ in range(nsteps):
        step_fn(ps, st)
    torch.cuda.synchronize()
    full = _packed(ps, st)
    for l, a in enumerate(start):
        st[l]["U"].copy_(torch.from_numpy(a))
    for _ in range(nsteps // 2):
        step_fn(ps, st)
    torch.cuda.synchronize()
    p = tmp_path / "run.safetensors"
    C.save(p, ps, st, t=0.5, step=nsteps // 2)
    ps2, st2, t, step, _ = C.restore(p)
    assert step == nsteps // 2 and t == 0.5
    for _ in range(nsteps - nsteps // 2):
        step_fn(ps2, st2)
    torch.cuda.synchronize()
    resumed = _packed(ps2, st2)
    for l in range(len(full)):
        assert np.all(np.isfinite(full[l])) or l > 0
        assert np.array_equal(full[l].view(np.uint64), resumed[l].view(np.uint64)), l


@pytest.mark.gpu
@pytest.mark.parametrize("system,nsteps", [(M.MOL_WAVE, 200), (M.MOL_CCZ4, 40)])
def test_restart_is_bitwise_on_the_ragged_hierarchy(tmp_path, system, nsteps):
    torch = _torch()
    from tests.test_gpu_amr import _setup
    print("checkpoint identity", system, nsteps, flush=True)
    ps, H, data, levels, dx0 = _setup(system)
    st = ps.alloc_states()
    for l, arrs in enumerate(data):
        st[l]["U"].copy_(torch.from_numpy(ps.pack(l, arrs)))
    dt0 = 0.25 * dx0
    _identity(tmp_path, ps, st, nsteps, lambda p, s: p.advance(s, dt0, M.MOL_BATCHED))


@pytest.mark.gpu
def test_restart_is_bitwise_for_brio_wu_with_fmr_ssprk3(tmp_path):
    torch = _torch()
    from paper_1806_04182_amd import mhd_runs as R
    from paper_1806_04182_amd import synth
    print("checkpoint identity brio-wu", flush=True)
    N = 50
    levels = R.brio_wu_levels(N, "2/2")
    sysd = M.System(M.MOL_MHD, sigma=0.0, gamma_ad=2.0)
    ps, st = R._run(levels, (int(R.BW_L * N), 1, 1), 1.0 / N, sysd, lambda n, h, lo: synth.mhd_brio_wu(n, h, lo),
                    R.BW_CFL_FMR / N, 0, ssp3=True)
    dt0 = R.BW_CFL_FMR / N
    _identity(tmp_path, ps, st, 100, lambda p, s: p.advance(s, dt0, M.MOL_BATCHED | M.MOL_ADV_SSPRK3))
