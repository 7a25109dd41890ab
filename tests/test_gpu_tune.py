"""Launch shapes and the autotuner: every shape gives the same results (the
split of work over the GPU never changes the arithmetic), and the autotuner
picks a shape from its candidate sets while the solve carries on."""
import numpy as np
import pytest

from paper_2511_07737_amd import gen, tsat

from parity_util import solver_or_skip

pytestmark = pytest.mark.gpu


def mixed_cnf():
    s = gen.structured(3000, 13000, seed=9)
    return s


def run(cnf_or_list, shape, steps=25, N=100, seed=4):
    s = solver_or_skip()
    if isinstance(cnf_or_list, list):
        s.load_batch(cnf_or_list)
    else:
        s.load(cnf_or_list)
    s.set_launch_config(**shape)
    s.init_batch(N, seed=seed)
    s.step(steps)
    th, m, v, t = s.get_state()
    bits = s.get_bits()
    s.close()
    return th, m, v, t, bits


SHAPES = [dict(fwd_target_blocks=256, var_blocks_per_cu=8, pure_group=1, clause_planes=0),
          dict(fwd_target_blocks=4096, var_blocks_per_cu=64, pure_group=4, clause_planes=0),
          dict(fwd_target_blocks=1000, var_blocks_per_cu=0, pure_group=2, clause_planes=1, window_gather=1),
          dict(fwd_target_blocks=777, var_blocks_per_cu=32, pure_group=2, clause_planes=1, window_gather=0),
          dict(fwd_target_blocks=512, var_blocks_per_cu=16, pure_group=2, clause_planes=0)]


@pytest.mark.parametrize("which", ["planted", "mixed", "batch"])
def test_results_do_not_depend_on_launch_shape(which):
    if which == "planted":
        cnf = gen.planted_ksat(2000, 8200, 3, seed=2)
    elif which == "mixed":
        cnf = mixed_cnf()
    else:
        cnf = [gen.planted_ksat(400 + 100 * j, 4 * (400 + 100 * j), 3, seed=30 + j) for j in range(5)]
    # a mixed-width store has two gathers that round differently: the clause
    # planes by windows, and the other literals' rows (planes off, or the
    # window gather off); shapes within each give identical results
    def gather(shape):
        if which != "mixed":
            return 0
        return int(shape.get("clause_planes", 1) == 1 and shape.get("window_gather", 1) == 1)

    refs = {}
    for shape in SHAPES:
        got = run(cnf, shape)
        ref = refs.setdefault(gather(shape), got)
        for a, b in zip(ref, got):
            assert np.array_equal(np.asarray(a), np.asarray(b))
    assert len(refs) == (2 if which == "mixed" else 1)


@pytest.mark.parametrize("pure", [True, False])
def test_autotune_picks_a_candidate_and_keeps_solving(pure):
    s = solver_or_skip()
    cnf = gen.planted_ksat(5000, 20500, 3, seed=3) if pure else mixed_cnf()
    s.load(cnf)
    s.init_batch(64, seed=1)
    before = s.launch_config()
    c, used = s.autotune(iters=2)
    assert c.fwd_target_blocks in (256, 512, 1024, 2048, 4096, 8192, 16384, 32768)
    assert c.var_blocks_per_cu in (0, 8, 16, 32, 64, 128, 256, 512, 1024)
    # the record group only matters (and is only tuned) for uniform-width stores
    assert c.pure_group in ((1, 2, 4) if pure else (before.pure_group,))
    assert c.fwd_ms > 0 and c.var_ms > 0
    assert c.clause_planes in (0, 1)
    # eight forward targets, then nine blocks per CU with the clause planes on (uniform
    # widths 2 and 3: by windows and by records; mixed: by windows) and, off,
    # with the three record groups (uniform widths only)
    assert used == 2 * (8 + (9 * 2 + 9 * 3 if pure else 9 + 9))
    got = s.launch_config()
    assert (got.fwd_target_blocks, got.var_blocks_per_cu, got.pure_group) == \
        (c.fwd_target_blocks, c.var_blocks_per_cu, c.pure_group)
    r = s.step(10)
    assert r.steps_done == 10
    _, _, _, t = s.get_state()
    assert t == used + 10
    s.close()


def test_launch_config_errors():
    s = solver_or_skip()
    for bad in (dict(fwd_target_blocks=0), dict(var_blocks_per_cu=-1), dict(pure_group=3), dict(clause_planes=2)):
        with pytest.raises(tsat.TsatError) as e:
            s.set_launch_config(**bad)
        assert e.value.code == tsat.E_ARG
    with pytest.raises(tsat.TsatError) as e:
        s.autotune(2)
    assert e.value.code == tsat.E_STATE
    s.close()
