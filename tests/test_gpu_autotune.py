"""Launch shapes and the autotuner: every shape gives the same hit set.

The shapes (child-phase LDS stage, wave-walker blocks per CU, lane-walker
waves per CU) change how the work is spread over the GPU, never which
states are computed, so the sorted hit set must be identical bit for bit; the
default shapes are pinned to the oracle by the parity tests, and here to the
oracle directly on a case that exercises every walker.
"""
import numpy as np
import pytest

import oracle
from paper_1208_0274_amd import alae, synth

pytestmark = pytest.mark.gpu

SHAPES = [dict(), dict(level_stage=2), dict(level_stage=8), dict(wide_blocks_per_cu=1),
          dict(wide_blocks_per_cu=6), dict(lane_waves_per_cu=2), dict(lane_waves_per_cu=16),
          dict(level_stage=8, wide_blocks_per_cu=2, lane_waves_per_cu=4)]


def homolog_case(seed, n=60000, m=600):
    rng = np.random.default_rng(seed)
    T = rng.integers(0, 4, size=n).astype(np.uint8)
    P = rng.integers(0, 4, size=m).astype(np.uint8)
    # long planted copies: wide rows for the wave walkers, gap states for the lane walker
    synth.plant_segments(rng, T, [P[40:520], P[100:300], P[:200]] * 2, 4, 0.08, 0.03)
    return T, P


def device_hits(ws):
    import torch

    k, s = ws.result_torch()
    torch.cuda.synchronize()
    return k.cpu().numpy().astype(np.int64), s.cpu().numpy().astype(np.int64)


@pytest.mark.parametrize("seed", [1, 2])
def test_shapes_same_hits(seed):
    import torch

    T, P = homolog_case(seed)
    idx = alae.Index.build(T, "dna")
    sc = alae.make_scoring(1, -3, -5, -2)
    H = 20
    ws = alae.Workspace(idx)
    dq = torch.from_numpy(P).to("cuda")
    ref = None
    for shape in SHAPES:
        st = alae.Stats()
        cnt = ws.search_device(dq, H, sc, stats=st, **shape)
        keys, scores = device_hits(ws)
        print(f"seed={seed} shape={shape} hits={cnt} wide_steps={st.wide_steps} chain_steps={st.chain_steps}",
              flush=True)
        if ref is None:
            ref = (keys, scores)
            assert st.wide_steps > 0 and st.chain_steps > 0  # both walkers ran
            # the default shapes against the oracle
            sub = oracle.scoring_table(4, 1, -3)
            qe, te, sv = oracle.sw_hits(T, P, sub, -5, -2, H, threads=8)
            np.testing.assert_array_equal(keys >> 32, qe)
            np.testing.assert_array_equal(keys & 0xFFFFFFFF, te)
            np.testing.assert_array_equal(scores, sv)
        else:
            np.testing.assert_array_equal(keys, ref[0], err_msg=str(shape))
            np.testing.assert_array_equal(scores, ref[1], err_msg=str(shape))
    ws.free()


def test_autotune_picks_valid_shapes():
    import torch

    T, P = homolog_case(3)
    idx = alae.Index.build(T, "dna")
    sc = alae.make_scoring(1, -3, -5, -2)
    H = 20
    ws = alae.Workspace(idx)
    dq = torch.from_numpy(P).to("cuda")
    base = ws.search_device(dq, H, sc)
    keys0, scores0 = device_hits(ws)
    shapes, rep = ws.autotune(dq, H, sc, reps=1)
    print(f"shapes={shapes} default_ms={rep['default_ms']:.3f} best_ms={rep['best_ms']:.3f} "
          f"trials={len(rep['trials'])}", flush=True)
    assert shapes["level_stage"] in (2, 4, 8)
    assert 1 <= shapes["wide_blocks_per_cu"] <= 8 and 1 <= shapes["lane_waves_per_cu"] <= 16
    assert shapes["level_graph"] in (0, 8)
    assert len(rep["trials"]) == 1 + 3 + 2 + 2 + 1  # the defaults, then every other candidate once
    assert 0 < rep["best_ms"] <= rep["default_ms"]
    cnt = ws.search_device(dq, H, sc, **shapes)
    keys, scores = device_hits(ws)
    assert cnt == base
    np.testing.assert_array_equal(keys, keys0)
    np.testing.assert_array_equal(scores, scores0)
    ws.free()
