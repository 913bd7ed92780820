"""Several CCD pairs in flight (PairPipeline over separate streams, handles
and workspaces; sfft_set_solve_team).

The kernels add in fixed orders, so a pair differenced in the pipeline must
equal, bit for bit, the same pair differenced alone with the same solve team.
A smaller team groups the solve's partial sums differently, so against the
default team the coefficients agree to rounding (checked at 1e-8 of their
largest magnitude), which ties the pipeline to the oracle parity of the
default path."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def _env():
    import torch
    import paper_2603_08593_amd as sf
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    sf.lib()
    return torch, sf


def test_solve_team_setting():
    torch, sf = _env()
    h = sf.Handle()
    try:
        assert sf.sfft_get_solve_team(h) == 0
        sf.sfft_set_solve_team(h, 32)
        assert sf.sfft_get_solve_team(h) == 32
        sf.sfft_set_solve_team(h, 0)
        assert sf.sfft_get_solve_team(h) == 0
        for bad in (-1, 1, 129):
            with pytest.raises(sf.SfftError):
                sf.sfft_set_solve_team(h, bad)
        assert sf.sfft_get_solve_team(h) == 0
    finally:
        h.close()


def _pairs(W, H, L, DK, DB, n, seed):
    if (W, H) == (2048, 4096):
        return [synth.make_cfg2(i) for i in range(n)]
    return [synth.make_pair(W, H, L, DK, DB, seed=seed + i, nstars=max(30, W * H // 1500), dtype=np.float32)
            for i in range(n)]


def _results(d):
    b = d.buf
    return (b.coef.cpu().numpy().copy(), b.diff.cpu().numpy().copy(), float(b.chi2.cpu()[0]), d.info().status)


@pytest.mark.parametrize("W,H,L,DK,DB,team,depth,rounds", [
    (256, 192, 7, 2, 1, 4, 3, 2),
    (2048, 4096, 11, 2, 2, 32, 3, 1),
])
def test_pipeline_matches_serial(W, H, L, DK, DB, team, depth, rounds):
    torch, sf = _env()
    _say(f"pipeline {W}x{H} L={L} DK={DK} DB={DB} team={team} depth={depth} rounds={rounds}")
    pairs = _pairs(W, H, L, DK, DB, depth, 9100)
    dev = [(torch.from_numpy(p.R).cuda(), torch.from_numpy(p.S).cuda()) for p in pairs]
    # serial references: one pair at a time, the same team and the default team
    ref_team, ref_default = [], []
    for t, out in ((team, ref_team), (0, ref_default)):
        d = sf.Differencer(W, H, L, DK, DB, solve_team=t)
        try:
            for R, S in dev:
                d.run(R, S, max_refine=1)
                torch.cuda.synchronize()
                out.append(_results(d))
        finally:
            d.close()
    pipe = sf.PairPipeline(W, H, L, DK, DB, depth=depth, solve_team=team)
    try:
        for rnd in range(rounds):
            # the pairs in reverse order in the second round, so every slot
            # is reused for a different pair
            order = list(range(depth)) if rnd % 2 == 0 else list(reversed(range(depth)))
            slots = {}
            for i in order:
                R, S = dev[i]
                slots[i] = pipe.submit(R, S, max_refine=1)
            pipe.wait()
            for i, k in slots.items():
                got = _results(pipe.slots[k])
                want = ref_team[i]
                assert got[3] == 0 and want[3] == 0
                assert np.array_equal(got[0], want[0]), f"pair {i}: coefficients differ from the serial run"
                assert np.array_equal(got[1], want[1]), f"pair {i}: difference image differs"
                assert got[2] == want[2], f"pair {i}: chi2 differs"
                dflt = ref_default[i]
                rel = np.max(np.abs(got[0] - dflt[0])) / np.max(np.abs(dflt[0]))
                _say(f"  round {rnd} pair {i} slot {k}: chi2 {got[2]:.6f}; team {team} vs default team: "
                     f"coef {rel:.2e} of max")
                assert rel <= 1e-8
                assert abs(got[2] - dflt[2]) <= 1e-9 * dflt[2]
    finally:
        pipe.close()
