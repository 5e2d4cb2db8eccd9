"""The FMR wave experiment (Sec. IV.A) on the GPU driver: channel runs with
each time-refinement strategy and with ratios 2, 4 and 2/2 against the
oracle's hierarchy step by step (states and the reflection integral Q), and
the convergence of Q measured on the GPU path at the paper's resolutions."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1806_04182_amd import fmr
from paper_1806_04182_amd import molamr as M
from paper_1806_04182_amd import synth
from tests.util import parity_err

pytestmark = pytest.mark.gpu

MODES = {M.MOL_TIME_BOR: O.TIME_BOR, M.MOL_TIME_BO: O.TIME_BO, M.MOL_TIME_BO1: O.TIME_BO1,
         M.MOL_TIME_NOSUB: O.TIME_NOSUB}


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU test needs a GPU"
    return torch


def _oracle_run(run, omode, t_end, window):
    """The oracle hierarchy with the same levels and data; Q after each step."""
    H = O.Hierarchy(O.WAVE, run.N0, (-2.0, 0.0, 0.0), run.dx0, run.levels)
    H.set_time_mode(omode)
    for l in range(len(run.levels)):
        H.set(l, 0, run.level_state(l)[0])
        H.fill_same(l)
    fine = run.dx0
    for R, _ in run.levels[1:]:
        fine /= R
    dt0 = 0.25 * (fine if omode == O.TIME_NOSUB else run.dx0)
    nsteps = int(round(t_end / dt0))
    x0 = -2.0 + np.arange(run.N0[0]) * run.dx0
    inside = (x0 >= -2.0) & (x0 <= -1.0)
    qs = []
    for s in range(nsteps):
        H.step(dt0, O.params(sigma=0.1))
        t = dt0 * (s + 1)
        if window[0] - 1e-12 <= t <= window[1] + 1e-12:
            qs.append(np.sum(np.abs(synth.interior(H.get(0, 0))[0, 0, 0][inside])) * run.dx0)
    return H, np.array(qs)


@pytest.mark.parametrize("tmode,ratios", [(M.MOL_TIME_BOR, (2,)), (M.MOL_TIME_BO, (2,)), (M.MOL_TIME_BO1, (2,)),
                                          (M.MOL_TIME_NOSUB, (2,)), (M.MOL_TIME_BOR, (4,)),
                                          (M.MOL_TIME_BOR, (2, 2)), (M.MOL_TIME_BO, (2, 2))])
def test_channel_run_matches_oracle(tmode, ratios):
    _torch()
    print("fmr channel", tmode, ratios, flush=True)
    run = fmr.ChannelRun(12, ratios)
    # the pulse's left half crosses [-2, -1] while the right half enters [1, 2]
    t_end, window = 1.5, (1.0, 1.5)
    H, q_ref = _oracle_run(run, MODES[tmode], t_end, window)
    q = run.run(t_end, tmode, window)
    assert q.shape == q_ref.shape and q.size > 0
    assert np.max(np.abs(q - q_ref)) <= 1e-12 * np.max(np.abs(q_ref)), (q, q_ref)
    for l in range(len(run.levels)):
        got = run.level_state(l)[0][:, 3:-3, 3:-3, 3:-3]
        ref = H.get(l, 0)[:, 3:-3, 3:-3, 3:-3]
        e = parity_err(got, ref)
        assert np.all(e <= 1e-12), (l, e)


def _orders(qs):
    q = np.array(qs)
    return np.log2(q[:-1] / q[1:])


def test_reflection_orders_at_paper_resolutions():
    """Coarse dx = 1/40, 1/80, 1/160: BOR and the run without sub-cycling
    reduce the reflections at 4th order, Berger-Oliger with the dense output
    only at 1st order, the linear Berger-Oliger at 1st order (Sec. IV.A)."""
    _torch()
    got = {}
    for tmode in (M.MOL_TIME_BOR, M.MOL_TIME_NOSUB, M.MOL_TIME_BO, M.MOL_TIME_BO1):
        got[tmode] = [fmr.reflection_q(n, tmode) for n in (40, 80, 160)]
        print("Q", tmode, got[tmode], _orders(got[tmode]), flush=True)
    assert _orders(got[M.MOL_TIME_BOR])[-1] > 3.5
    assert _orders(got[M.MOL_TIME_NOSUB])[-1] > 3.5
    assert 0.6 < _orders(got[M.MOL_TIME_BO])[-1] < 1.5
    assert 0.6 < _orders(got[M.MOL_TIME_BO1])[-1] < 1.5
    # the finest BOR reflections are far below the BO ones and close to the
    # run without sub-cycling
    assert got[M.MOL_TIME_BOR][-1] < got[M.MOL_TIME_BO][-1] / 10
    assert got[M.MOL_TIME_BOR][-1] < 3 * got[M.MOL_TIME_NOSUB][-1]


def test_ratio4_and_ratio22_reflections_are_similar():
    """One level of ratio 4 against two levels of ratio 2 (Sec. IV.A): with
    BOR the reflections are of the same size, slightly larger with ratio 4;
    at the finest resolution both are far below those of BO."""
    _torch()
    q4 = fmr.reflection_q(80, M.MOL_TIME_BOR, ratios=(4,))
    q22 = fmr.reflection_q(80, M.MOL_TIME_BOR, ratios=(2, 2))
    print("Q ratio 4", q4, "ratio 2/2", q22, flush=True)
    assert 1.0 < q4 / q22 < 2.0
    for ratios in ((4,), (2, 2)):
        bor = fmr.reflection_q(160, M.MOL_TIME_BOR, ratios=ratios)
        bo = fmr.reflection_q(160, M.MOL_TIME_BO, ratios=ratios)
        print("Q 1/160", ratios, "BOR", bor, "BO", bo, flush=True)
        assert bor < bo / 5
