"""Host-side checks of the C ABI: the library loads, exports every entry
point include/ga.h declares, and rejects invalid configurations (no GPU
work is launched here)."""
import ctypes
import os
import re

import pytest

import paper_2208_14961_amd as ga

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "ga.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ga_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    names = declared_functions()
    assert len(names) >= 15
    L = ctypes.CDLL(ga.LIB_PATH)
    for name in names:
        assert hasattr(L, name), name


def test_population_words():
    assert ga.ga_population_words(ga.Config(m=20, n=40000)) == 40000 * 20
    assert ga.ga_population_words(ga.Config(m=36, n=10)) == 10 * 36 * 2
    assert ga.ga_population_words(ga.Config(m=64, n=3)) == 3 * 64 * 2
    assert ga.ga_population_words(ga.Config(m=68, n=3)) == 3 * 68 * 4
    assert ga.ga_population_words(ga.Config(m=100, n=40000)) == 40000 * 100 * 4
    assert ga.ga_population_words(ga.Config(m=128, n=5)) == 5 * 128 * 4
    assert ga.ga_population_words(ga.Config(m=6, n=3)) == 0
    assert ga.ga_population_words(ga.Config(m=132, n=3)) == 0


@pytest.mark.parametrize("kw", [
    dict(m=6), dict(m=0), dict(m=132), dict(n=1), dict(n=(1 << 24) + 1), dict(fitness=6),
    dict(selection=2), dict(tournament_k=0), dict(tournament_k=65), dict(elite=10),
    dict(xo_threshold=(1 << 32) + 1), dict(mut_threshold=(1 << 32) + 1), dict(nc=0),
    dict(nr=0), dict(nc=65), dict(flags=4), dict(selection=ga.SEL_PAPER, n=10),
    dict(selection=ga.SEL_PAPER, n=12, elite=1),
    dict(flags=ga.lanes_flag(3)), dict(flags=ga.lanes_flag(1)), dict(flags=ga.lanes_flag(16)),
    dict(m=36, flags=ga.lanes_flag(2)), dict(m=68, flags=ga.lanes_flag(4)),
    dict(m=128, flags=ga.lanes_flag(2)), dict(m=64, flags=ga.lanes_flag(16)),
    dict(m=128, flags=ga.lanes_flag(31)),
    # keys that elitism and paper selection cannot rank (the SQ keys reach
    # C(m-1, 2) m^2 >= 2^24 from order 80 on)
    dict(m=80, n=100, elite=1), dict(m=80, n=100, elite=1, fitness=ga.FIT_SQ_PLUS_NNZ),
    dict(m=128, n=400, selection=ga.SEL_PAPER, fitness=ga.FIT_SQ),
    # generation budgets whose generation numbers could pass 2^32
    dict(max_generations=1 << 31), dict(max_generations=(1 << 32) - 1),
    # the matrix-core Gram path starts at order 36; both Gram flags at once
    dict(m=32, flags=ga.GRAM_MFMA), dict(m=64, flags=ga.GRAM_MFMA | ga.GRAM_PACKED),
])
def test_invalid_configs(kw):
    base = dict(m=8, n=10)
    cfg = ga.Config(**{**base, **kw})
    assert not ga.ga_validate(cfg)
    assert ga.lib().ga_last_error().decode() != ""


def test_valid_configs():
    for cfg in [ga.Config(m=8, n=10), ga.Config(m=64, n=2, elite=1),
                ga.Config(m=20, n=40000, fitness=ga.FIT_ABS),
                ga.Config(m=32, n=200000, elite=2000, fitness=ga.FIT_SQ_PLUS_NNZ),
                ga.Config(m=12, n=4000, selection=ga.SEL_PAPER, fitness=ga.FIT_F2,
                          xo_threshold=1 << 32, mut_threshold=1 << 32, nc=1, nr=2),
                ga.Config(m=8, n=10, mut_threshold=0, nc=0, nr=0),
                ga.Config(m=8, n=10, flags=ga.lanes_flag(2)),
                ga.Config(m=32, n=10, flags=ga.STOP_ON_FOUND | ga.lanes_flag(8)),
                ga.Config(m=64, n=10, flags=ga.lanes_flag(4)),
                ga.Config(m=12, n=40, flags=ga.MUT_SHARED | ga.STOP_ON_FOUND),
                ga.Config(m=68, n=10, flags=ga.lanes_flag(16)),
                ga.Config(m=128, n=10, flags=ga.lanes_flag(8)),
                ga.Config(m=128, n=10),  # tournaments take every kind
                ga.Config(m=76, n=100, elite=1), ga.Config(m=76, n=100, elite=1,
                                                          fitness=ga.FIT_SQ_PLUS_NNZ),
                ga.Config(m=128, n=100, elite=1, fitness=ga.FIT_ABS),
                ga.Config(m=100, n=40000, selection=ga.SEL_PAPER, fitness=ga.FIT_F1,
                          xo_threshold=1 << 32, mut_threshold=1 << 32, nc=4, nr=2),
                ga.Config(m=8, n=10, max_generations=(1 << 31) - 1),
                ga.Config(m=36, n=10, flags=ga.GRAM_MFMA), ga.Config(m=128, n=10, flags=ga.GRAM_MFMA),
                ga.Config(m=8, n=10, flags=ga.GRAM_PACKED)]:
        assert ga.ga_validate(cfg), cfg


def test_binding_rejects_host_tensors():
    import torch
    cfg = ga.Config(m=8, n=10)
    with pytest.raises(TypeError):
        ga.ga_init_population(cfg, torch.zeros((10, 8, 1), dtype=torch.int32))


def test_fitness_repeat_rejects_bad_repeat_counts():
    """Argument checks run before any device work: no GPU is touched."""
    L = ga.lib()
    cfg = ga.Config(m=20, n=40000).c()
    fake = ctypes.c_void_p(256)            # never dereferenced: rejected first
    assert L.ga_fitness_repeat(ctypes.byref(cfg), fake, fake, 0, None) == ga.GA_EINVAL
    assert "reps" in L.ga_last_error().decode()
    assert L.ga_fitness_repeat(ctypes.byref(cfg), fake, fake, 1 << 30, None) == ga.GA_EINVAL
    assert L.ga_fitness_repeat(ctypes.byref(cfg), None, fake, 5, None) == ga.GA_EINVAL


def test_pack_unpack_reject_bad_arguments():
    """Argument checks run before any device work: no GPU is touched."""
    L = ga.lib()
    fake = ctypes.c_void_p(256)            # never dereferenced: rejected first
    good = ga.Config(m=20, n=10).c()
    assert L.ga_pack(ctypes.byref(good), None, fake, None, None) == ga.GA_EINVAL
    assert L.ga_pack(ctypes.byref(good), fake, None, None, None) == ga.GA_EINVAL
    assert L.ga_unpack(ctypes.byref(good), None, fake, None) == ga.GA_EINVAL
    assert L.ga_unpack(ctypes.byref(good), fake, None, None) == ga.GA_EINVAL
    bad = ga.Config(m=132, n=10).c()
    assert L.ga_pack(ctypes.byref(bad), fake, fake, None, None) == ga.GA_EINVAL
    assert L.ga_unpack(ctypes.byref(bad), fake, fake, None) == ga.GA_EINVAL


def test_batch_rejects_invalid_runs_before_device_work():
    """ga_run_batch validates every config first (paper mode and elitism are
    accepted, an invalid run is not), and needs results to write."""
    L = ga.lib()
    cfgs = (ga._Config * 2)(ga.Config(m=12, n=400, selection=ga.SEL_PAPER).c(),
                            ga.Config(m=18, n=100).c())
    outs = (ga._Result * 2)()
    assert L.ga_run_batch(cfgs, 2, outs, None) == ga.GA_EINVAL
    assert "m=18" in L.ga_last_error().decode()
    assert L.ga_run_batch(cfgs, 0, outs, None) == ga.GA_EINVAL
    assert L.ga_run_batch(cfgs, 2, None, None) == ga.GA_EINVAL


def test_tuning_table_is_well_formed():
    """The committed lanes-per-child table: one row per order, allowed
    lanes only, increasing size limits with an open last entry."""
    import re
    path = os.path.join(os.path.dirname(ga.LIB_PATH), "csrc", "ga_tuned.h")
    text = open(path).read()
    sizes = int(re.search(r"kTuneSizes = (\d+);", text).group(1))
    limits = re.search(r"kTuneMaxChildren\[kTuneSizes\] = \{([^}]*)\}", text).group(1)
    limits = [x.strip() for x in limits.split(",")]
    assert len(limits) == sizes and limits[-1] == "~0ull"
    nums = [int(x) for x in limits[:-1]]
    assert nums == sorted(nums) and len(set(nums)) == len(nums)
    rows = re.findall(r"^\s*\{([0-9, ]+)\},\s*// m = (\d+)", text, re.M)
    assert [int(m) for _, m in rows] == list(range(4, ga.MAX_ORDER + 1, 4))
    for cells, m in rows:
        lanes = [int(x) for x in cells.split(",")]
        assert len(lanes) == sizes
        allowed = {2, 4, 8} if int(m) <= 32 else ({4, 8} if int(m) <= 64 else {8, 16})
        assert set(lanes) <= allowed, (m, lanes)


def test_tuned_lanes_query():
    """Forced lanes are returned as given; otherwise an allowed value."""
    assert ga.ga_tuned_lanes(ga.Config(m=8, n=100, flags=ga.lanes_flag(2))) == 2
    assert ga.ga_tuned_lanes(ga.Config(m=20, n=40000)) in (2, 4, 8)
    assert ga.ga_tuned_lanes(ga.Config(m=64, n=50000)) in (4, 8)
    assert ga.ga_tuned_lanes(ga.Config(m=100, n=40000)) in (8, 16)
    assert ga.ga_tuned_lanes(ga.Config(m=128, n=40000, flags=ga.lanes_flag(8))) == 8
    assert ga.ga_tuned_lanes(ga.Config(m=6, n=100)) == 0


def test_run_rejects_unbounded_budget_before_device_work():
    """A budget of 2^32 - 1 generations (a natural 'until found' value) is
    rejected by ga_run itself before any device work, instead of wrapping
    its chunk count."""
    L = ga.lib()
    fake = ctypes.c_void_p(256)            # never dereferenced: rejected first
    cfg = ga.Config(m=8, n=10, max_generations=(1 << 32) - 1).c()
    out = ga._Result()
    assert L.ga_run(ctypes.byref(cfg), fake, ctypes.c_void_p(512), fake,
                    ctypes.c_void_p(512), ctypes.byref(out), None) == ga.GA_EINVAL
    assert "max_generations" in L.ga_last_error().decode()


def test_paper_select_rejects_bad_arguments_before_device_work():
    """ga_paper_select takes paper-mode configs up to 65,536 individuals and
    non-NULL buffers; it checks before any device work."""
    L = ga.lib()
    fake = ctypes.c_void_p(256)  # never dereferenced
    paper = ga.Config(m=20, n=40000, selection=ga.SEL_PAPER, fitness=ga.FIT_F2).c()
    tour = ga.Config(m=20, n=40000).c()
    big = ga.Config(m=20, n=65540, selection=ga.SEL_PAPER, fitness=ga.FIT_F2).c()
    assert L.ga_paper_select(ctypes.byref(tour), fake, fake, fake, None) == ga.GA_EINVAL
    assert L.ga_paper_select(ctypes.byref(big), fake, fake, fake, None) == ga.GA_EINVAL
    assert "65536" in L.ga_last_error().decode()
    assert L.ga_paper_select(ctypes.byref(paper), None, fake, fake, None) == ga.GA_EINVAL
    assert L.ga_paper_select(ctypes.byref(paper), fake, None, fake, None) == ga.GA_EINVAL
    assert L.ga_paper_select(ctypes.byref(paper), fake, fake, None, None) == ga.GA_EINVAL
