"""GPU-vs-oracle parity of every entry point of libga.  All results are
integers and must match bit for bit."""
import zlib

import numpy as np
import pytest

import paper_2208_14961_amd as ga
from oracle import gao
from tests import hadamard_fixtures as hf
from tests import inputs
from tests.gpu_util import (announce, dev_pop_from_int8, empty_keys, empty_pop,
                            int8_from_dev_pop, keys_np, to_oracle, torch_cuda)

pytestmark = pytest.mark.gpu

ORDERS = list(range(4, ga.MAX_ORDER + 1, 4))
WIDE_SQ = (ga.FIT_SQ, ga.FIT_SQ_PLUS_NNZ)  # keys elitism cannot rank from order 80 on


def lanes_of(m):
    return (2, 4, 8) if m <= 32 else ((4, 8) if m <= 64 else (8, 16))
KINDS = [ga.FIT_SQ, ga.FIT_ABS, ga.FIT_NNZ, ga.FIT_SQ_PLUS_NNZ, ga.FIT_F1, ga.FIT_F2]


# --------------------------------------------------------------------------
# Gram + fitness
# --------------------------------------------------------------------------
@pytest.mark.parametrize("m", ORDERS)
def test_fitness_random_all_kinds(m):
    torch = torch_cuda()
    n = 3 * 256 + 37                       # several blocks and a ragged tail
    announce("fitness", m, n)
    pop = inputs.random_population(m, n, seed=100 + m)
    dpop = dev_pop_from_int8(pop)
    # the library's choice of Gram path, and the popcount path forced where
    # the table picks the matrix cores
    grams = [0] if m < ga.MFMA_MIN_ORDER else [0, ga.GRAM_PACKED]
    for kind in KINDS:
        for gram in grams:
            cfg = ga.Config(m=m, n=n, fitness=kind, flags=gram)
            keys = empty_keys(cfg)
            comps = torch.zeros((n, 3), dtype=torch.int32, device="cuda")
            ga.ga_fitness(cfg, dpop, keys, comps)
            want, want_c = gao.fitness(to_oracle(cfg), pop, with_comps=True)
            assert np.array_equal(keys_np(keys), want), (kind, gram)
            assert np.array_equal(comps.cpu().numpy().view(np.uint32), want_c)
            keys2 = empty_keys(cfg)
            ga.ga_fitness(cfg, dpop, keys2)    # without components
            assert np.array_equal(keys_np(keys2), want)


@pytest.mark.parametrize("m", ORDERS)
def test_fitness_repeat_equals_oracle(m):
    """The repeated whole-population evaluation writes the same keys as one
    evaluation, for every order, kind and a ragged n."""
    torch_cuda()
    n = 2 * 256 + 91
    announce("fitness repeat", m, n)
    pop = inputs.random_population(m, n, seed=300 + m)
    dpop = dev_pop_from_int8(pop)
    grams = [0] if m < ga.MFMA_MIN_ORDER else [0, ga.GRAM_PACKED]
    for i, kind in enumerate(KINDS):
        for gram in grams:
            cfg = ga.Config(m=m, n=n, fitness=kind, flags=gram)
            keys = empty_keys(cfg)
            ga.ga_fitness_repeat(cfg, dpop, keys, reps=1 + 2 * (i % 3))
            want = gao.fitness(to_oracle(cfg), pop)
            assert np.array_equal(keys_np(keys), want), (kind, gram)


def test_fitness_repeat_full_size_m20_n40000():
    """The kernel-metric configuration: m=20, n=40,000, SQ and ABS keys of
    the seed-1 initial population, evaluated 1000 times."""
    torch_cuda()
    announce("fitness repeat m20 n40000")
    for kind in (ga.FIT_SQ, ga.FIT_ABS):
        cfg = ga.Config(m=20, n=40000, seed=1, fitness=kind)
        dpop = empty_pop(cfg)
        ga.ga_init_population(cfg, dpop)
        keys = empty_keys(cfg)
        ga.ga_fitness_repeat(cfg, dpop, keys, reps=1000)
        want = gao.fitness(to_oracle(cfg), int8_from_dev_pop(dpop, cfg.m))
        assert np.array_equal(keys_np(keys), want), kind
        opop = gao.init_population(to_oracle(cfg))
        assert np.array_equal(int8_from_dev_pop(dpop, cfg.m), opop)


def test_fitness_known_hadamard_and_census():
    torch_cuda()
    for m in hf.ORDERS_WITH_FIXTURE:
        announce("hadamard fixture", m)
        H = hf.hadamard(m)
        # the fixture among random matrices, at a ragged position
        pop = inputs.random_population(m, 300, seed=m)
        pop[257] = H
        cfg = ga.Config(m=m, n=300, fitness=ga.FIT_F2)
        keys = empty_keys(cfg)
        ga.ga_fitness(cfg, dev_pop_from_int8(pop), keys)
        k = keys_np(keys)
        assert k[257] == 0 and np.count_nonzero(k == 0) >= 1
        assert np.array_equal(k, gao.fitness(to_oracle(cfg), pop))
    announce("m4 census")
    pops = inputs.all_m4_normalized()
    cfg = ga.Config(m=4, n=len(pops), fitness=ga.FIT_SQ)
    keys = empty_keys(cfg)
    ga.ga_fitness(cfg, dev_pop_from_int8(pops), keys)
    vals, counts = np.unique(keys_np(keys), return_counts=True)
    assert dict(zip(vals.tolist(), counts.tolist())) == {0: 48, 16: 144, 48: 24}


@pytest.mark.parametrize("m", [8, 20, 32, 36, 64, 68, 100, 128])
def test_fitness_all_equal_columns(m):
    torch_cuda()
    announce("all-equal", m)
    Q = np.ones((m, m), dtype=np.int8)
    Q[: m // 2, 1:] = -1
    pop = np.stack([Q] * 5)
    P = (m - 1) * (m - 2) // 2
    for kind, want in [(ga.FIT_SQ, P * m * m), (ga.FIT_ABS, P * m), (ga.FIT_NNZ, P),
                       (ga.FIT_SQ_PLUS_NNZ, P * m * m + P), (ga.FIT_F1, 2 * P * m),
                       (ga.FIT_F2, 2 * P)]:
        cfg = ga.Config(m=m, n=5, fitness=kind)
        keys = empty_keys(cfg)
        ga.ga_fitness(cfg, dev_pop_from_int8(pop), keys)
        assert (keys_np(keys) == want).all()


# --------------------------------------------------------------------------
# Gram products on the matrix cores (int8 MFMA), orders 36..128
# --------------------------------------------------------------------------
MFMA_ORDERS = [m for m in ORDERS if m >= ga.MFMA_MIN_ORDER]


@pytest.mark.parametrize("m", MFMA_ORDERS)
def test_fitness_mfma_all_kinds(m):
    """The matrix-core Gram path gives the oracle's keys and components for
    every kind, over several waves' worth of individuals and a ragged
    count, in the single and the repeated form."""
    torch = torch_cuda()
    n = 2 * 256 + 37
    announce("fitness mfma", m, n)
    pop = inputs.random_population(m, n, seed=1100 + m)
    dpop = dev_pop_from_int8(pop)
    for i, kind in enumerate(KINDS):
        cfg = ga.Config(m=m, n=n, fitness=kind, flags=ga.GRAM_MFMA)
        keys = empty_keys(cfg)
        comps = torch.zeros((n, 3), dtype=torch.int32, device="cuda")
        ga.ga_fitness(cfg, dpop, keys, comps)
        want, want_c = gao.fitness(to_oracle(cfg), pop, with_comps=True)
        assert np.array_equal(keys_np(keys), want), kind
        assert np.array_equal(comps.cpu().numpy().view(np.uint32), want_c)
        keys2 = empty_keys(cfg)
        ga.ga_fitness(cfg, dpop, keys2)
        assert np.array_equal(keys_np(keys2), want), kind
        keys3 = empty_keys(cfg)
        ga.ga_fitness_repeat(cfg, dpop, keys3, reps=1 + i % 3)
        assert np.array_equal(keys_np(keys3), want), kind


def test_fitness_mfma_hadamard_and_closed_form():
    """Hadamard matrices have key 0 on the matrix-core path, and a matrix of
    equal columns has the closed-form keys (every pair |G| = m)."""
    torch_cuda()
    for m in [x for x in hf.ORDERS_WITH_FIXTURE if x >= ga.MFMA_MIN_ORDER]:
        announce("mfma hadamard", m)
        pop = inputs.random_population(m, 70, seed=m)
        pop[33] = hf.hadamard(m)
        cfg = ga.Config(m=m, n=70, fitness=ga.FIT_F2, flags=ga.GRAM_MFMA)
        keys = empty_keys(cfg)
        ga.ga_fitness(cfg, dev_pop_from_int8(pop), keys)
        k = keys_np(keys)
        assert k[33] == 0 and np.array_equal(k, gao.fitness(to_oracle(cfg), pop))
    for m in (36, 64, 68, 100, 128):
        Q = np.ones((m, m), dtype=np.int8)
        Q[: m // 2, 1:] = -1
        P = (m - 1) * (m - 2) // 2
        for kind, want in [(ga.FIT_SQ, P * m * m), (ga.FIT_ABS, P * m), (ga.FIT_NNZ, P)]:
            cfg = ga.Config(m=m, n=3, fitness=kind, flags=ga.GRAM_MFMA)
            keys = empty_keys(cfg)
            ga.ga_fitness(cfg, dev_pop_from_int8(np.stack([Q] * 3)), keys)
            assert (keys_np(keys) == want).all(), (m, kind)


# --------------------------------------------------------------------------
# Layout conversion
# --------------------------------------------------------------------------
@pytest.mark.parametrize("m", [4, 20, 32, 36, 64, 68, 96, 100, 128])
def test_pack_unpack(m):
    """The paper's int8 layout to the packed one and back: the packed words
    equal the layout's definition (computed on the host by tests/inputs),
    the round trip is the identity, and entries other than +1/-1 are
    counted (packing as -1 iff negative)."""
    torch = torch_cuda()
    n = 257
    announce("pack", m, n)
    pop = inputs.random_population(m, n, seed=900 + m)
    cfg = ga.Config(m=m, n=n)
    q = torch.from_numpy(pop).to("cuda")
    packed = empty_pop(cfg)
    bad = torch.zeros((1,), dtype=torch.int32, device="cuda")
    ga.ga_pack(cfg, q, packed, bad)
    assert np.array_equal(packed.cpu().numpy().view(np.uint32), inputs.pack(pop))
    assert int(bad.item()) == 0 and ga.ga_check_invariants(cfg, packed) == 0
    back = torch.zeros_like(q)
    ga.ga_unpack(cfg, packed, back)
    assert np.array_equal(back.cpu().numpy(), pop)
    odd = pop.copy()
    rng = np.random.default_rng(m)
    at = rng.integers(0, n * m * m, 40)
    flat = odd.reshape(-1)
    flat[at] = rng.choice(np.array([0, 2, -3, 5, -128], dtype=np.int8), 40)
    ga.ga_pack(cfg, torch.from_numpy(odd).to("cuda"), packed, bad)
    assert int(bad.item()) == len(set(at.tolist()))
    assert np.array_equal(packed.cpu().numpy().view(np.uint32),
                          inputs.pack(np.where(odd < 0, -1, 1).astype(np.int8)))


# --------------------------------------------------------------------------
# Initial population
# --------------------------------------------------------------------------
@pytest.mark.parametrize("m", ORDERS)
def test_init_parity(m):
    torch_cuda()
    for n, seed in [(1, 0), (257, 5), (1000, (7 << 32) | 3)]:
        if n < 2:
            continue
        announce("init", m, n, seed)
        cfg = ga.Config(m=m, n=n, seed=seed)
        pop = empty_pop(cfg)
        ga.ga_init_population(cfg, pop)
        got = int8_from_dev_pop(pop, m)
        assert np.array_equal(got, gao.init_population(to_oracle(cfg)))
        assert ga.ga_check_invariants(cfg, pop) == 0


# --------------------------------------------------------------------------
# Steps
# --------------------------------------------------------------------------
def _step_chain(cfg: ga.Config, gens: int, start=None):
    """Runs `gens` steps on the GPU and on the oracle from the same start;
    compares every generation."""
    ocfg = to_oracle(cfg)
    pop = gao.init_population(ocfg) if start is None else start
    keys = gao.fitness(ocfg, pop)
    dpop, dkeys = dev_pop_from_int8(pop), empty_keys(cfg)
    ga.ga_fitness(cfg, dpop, dkeys)
    assert np.array_equal(keys_np(dkeys), keys)
    nxt_pop, nxt_keys = empty_pop(cfg), empty_keys(cfg)
    for g in range(gens):
        ga.ga_step(cfg, dpop, dkeys, nxt_pop, nxt_keys, g)
        pop, keys = gao.step(ocfg, pop, keys, g)
        got = int8_from_dev_pop(nxt_pop, cfg.m)
        assert np.array_equal(keys_np(nxt_keys), keys), f"keys differ at gen {g + 1}"
        assert np.array_equal(got, pop), f"population differs at gen {g + 1}"
        assert ga.ga_check_invariants(cfg, nxt_pop) == 0
        dpop, nxt_pop = nxt_pop, dpop
        dkeys, nxt_keys = nxt_keys, dkeys


@pytest.mark.parametrize("m", ORDERS)
def test_step_tournament(m):
    torch_cuda()
    n = 2 * 256 + 77
    announce("step tournament", m, n)
    cfg = ga.Config(m=m, n=n, seed=m, mut_threshold=ga.rate_threshold(1, 2), nc=2, nr=3)
    _step_chain(cfg, 3)


LANES = [(m, L) for m in ORDERS for L in lanes_of(m)]


@pytest.mark.parametrize("m,lanes", LANES)
def test_step_lanes(m, lanes):
    """Every lanes-per-child variant of the children kernel gives the
    oracle's generation (the tile shape never changes a result)."""
    torch_cuda()
    n = 2 * 128 + 45
    announce("step lanes", m, lanes, n)
    kind = KINDS[(m // 4 + lanes) % len(KINDS)]
    cfg = ga.Config(m=m, n=n, seed=500 + m + lanes,
                    elite=0 if (m >= 80 and kind in WIDE_SQ) else m % 3, fitness=kind,
                    mut_threshold=ga.rate_threshold(1, 2), nc=1 + lanes % 3, nr=1 + m % 2,
                    flags=ga.lanes_flag(lanes))
    _step_chain(cfg, 2)


@pytest.mark.parametrize("m,n,t,elite,kind", [
    (8, 1024, 2, 0, ga.FIT_SQ),
    (12, 999, 3, 7, ga.FIT_NNZ),
    (20, 1001, 1, 0, ga.FIT_ABS),
    (28, 700, 5, 69, ga.FIT_SQ_PLUS_NNZ),
    (32, 3000, 2, 30, ga.FIT_SQ_PLUS_NNZ),
    (44, 513, 4, 100, ga.FIT_F1),
    (64, 300, 2, 3, ga.FIT_F2),
    (68, 301, 2, 4, ga.FIT_SQ_PLUS_NNZ),
    (100, 333, 2, 5, ga.FIT_F1),
    (128, 257, 3, 0, ga.FIT_SQ),
    (124, 190, 2, 9, ga.FIT_NNZ),
])
def test_step_variants(m, n, t, elite, kind):
    torch_cuda()
    announce("step variant", m, n, t, elite, kind)
    cfg = ga.Config(m=m, n=n, seed=11, tournament_k=t, elite=elite, fitness=kind,
                    xo_threshold=ga.rate_threshold(3, 4), mut_threshold=ga.rate_threshold(1, 3),
                    nc=3, nr=2)
    _step_chain(cfg, 4)


@pytest.mark.parametrize("m,n,elite,paper", [
    (8, 2_200_001, 30_000, False),     # more than 1024 selection tiles
    (4, 4 * 600_000, 0, True),
])
def test_step_selection_many_tiles(m, n, elite, paper):
    """Selection over more than 1024 tiles of 512 keys takes the unfused
    pipeline (separate threshold and offset launches)."""
    torch_cuda()
    announce("step many tiles", m, n, elite, paper)
    if paper:
        cfg = ga.Config(m=m, n=n, seed=13, selection=ga.SEL_PAPER, fitness=ga.FIT_F2,
                        xo_threshold=1 << 32, mut_threshold=1 << 32, nc=1, nr=1)
    else:
        cfg = ga.Config(m=m, n=n, seed=12, elite=elite, fitness=ga.FIT_SQ)
    _step_chain(cfg, 2)


def test_step_elite_with_ties():
    """Many equal keys: the elite set breaks ties by index."""
    torch_cuda()
    m, n = 8, 600
    announce("elite ties", m, n)
    H = hf.hadamard(8)
    pop = inputs.random_population(m, n, seed=2)
    pop[::3] = H                           # 200 copies with key 0
    cfg = ga.Config(m=m, n=n, seed=4, elite=150, flags=0)
    _step_chain(cfg, 3, start=pop)


def _paper_select_case(name, n):
    """Keys of one generation and a starting threshold (None: none known)."""
    rng = np.random.default_rng(zlib.crc32(name.encode()))
    D = n // 2
    if name == "oracle_gen0":  # the initial keys of the m = 20 Table 2 run
        cfg = gao.Config(m=20, n=n, seed=9020, selection=gao.SEL_PAPER, fitness=gao.FIT_F2)
        return gao.fitness(cfg, gao.init_population(cfg)), None
    if name.startswith("spread"):
        keys = rng.integers(100_000, 300_000, n).astype(np.uint32)
    elif name == "ties":
        keys = rng.integers(0, 50, n).astype(np.uint32)
    elif name == "all_equal":
        keys = np.full(n, 77, dtype=np.uint32)
    else:
        keys = rng.integers(0, 5000, n).astype(np.uint32)
    T = int(np.sort(keys)[D - 1])
    prev = {"spread_below_window": T + 1000,     # keys below the 16-bit window
            "spread_window_missed": T + 100_000,  # T below the window: the slow path
            "spread_unaligned": T + 300,
            "ties": 60, "all_equal": 77, "prev_is_T": T, "prev_above": T + 37,
            "cold": None}[name]
    return keys, prev


@pytest.mark.parametrize("name,n", [
    ("oracle_gen0", 40000), ("cold", 4), ("cold", 400), ("prev_is_T", 1028),
    ("prev_above", 40000), ("spread_below_window", 4096), ("spread_below_window", 65536),
    ("spread_window_missed", 40000), ("spread_unaligned", 40000), ("ties", 40000),
    ("ties", 65536), ("all_equal", 2052), ("cold", 65536),
])
def test_paper_select(name, n):
    """The tile truncation selection (Sec. 3.3) of ga_run's paper mode on its
    own: threshold and selected set against the oracle's selection of the n/2
    smallest (key, index), from a cold start, from thresholds at or above the
    answer, with keys below the 1024-value window it counts in, with the
    answer below that window, and with long runs of equal keys."""
    torch = torch_cuda()
    announce("paper select", name, n)
    keys, prev = _paper_select_case(name, n)
    D = n // 2
    # order 64, SQ: keys up to 8,000,256, above every key drawn here
    cfg = ga.Config(m=64, n=n, seed=1, selection=ga.SEL_PAPER, fitness=ga.FIT_SQ)
    kd = torch.from_numpy(keys.view(np.int32).copy()).cuda()
    if name == "spread_unaligned":  # keys at a 4-byte offset: the scalar tile loads
        kd = torch.cat([torch.zeros(1, dtype=torch.int32, device="cuda"), kd])[1:]
    sel = torch.full((D,), -7, dtype=torch.int32, device="cuda")
    thr = torch.tensor([-1 if prev is None else prev], dtype=torch.int32, device="cuda")
    ga.ga_paper_select(cfg, kd, thr, sel)
    assert int(keys_np(thr)[0]) == int(np.sort(keys)[D - 1])
    assert np.array_equal(keys_np(sel), np.sort(gao.select_set(keys, D)))


@pytest.mark.parametrize("m,N,nc,nr,kind", [
    (12, 250, 1, 2, ga.FIT_F2), (20, 100, 4, 2, ga.FIT_F1), (16, 1, 2, 2, ga.FIT_F2),
    (40, 64, 2, 8, ga.FIT_F2), (8, 4096, 3, 2, ga.FIT_F2),
    (100, 250, 4, 2, ga.FIT_F2), (128, 33, 1, 1, ga.FIT_F1), (76, 40, 3, 5, ga.FIT_SQ),
])
def test_step_paper_mode(m, N, nc, nr, kind):
    torch_cuda()
    announce("step paper", m, N, nc, nr)
    cfg = ga.Config(m=m, n=4 * N, seed=21, selection=ga.SEL_PAPER, fitness=kind,
                    xo_threshold=1 << 32, mut_threshold=1 << 32, nc=nc, nr=nr)
    _step_chain(cfg, 3)


# --------------------------------------------------------------------------
# Whole runs
# --------------------------------------------------------------------------
@pytest.mark.parametrize("m,lanes,paper", [(12, 4, True), (20, 2, False), (44, 8, True),
                                           (64, 4, False), (100, 16, True), (128, 8, False)])
def test_step_shared_mutation(m, lanes, paper):
    """The first mutation method (one draw set per generation, shared by
    every mutated child) in every column width and tile shape family."""
    torch_cuda()
    announce("step shared mutation", m, lanes, paper)
    if paper:
        cfg = ga.Config(m=m, n=4 * 61, seed=40 + m, selection=ga.SEL_PAPER, fitness=ga.FIT_F2,
                        xo_threshold=1 << 32, mut_threshold=1 << 32, nc=1, nr=1,
                        flags=ga.MUT_SHARED | ga.lanes_flag(lanes))
    else:
        cfg = ga.Config(m=m, n=2 * 128 + 45, seed=41 + m, elite=3, fitness=ga.FIT_ABS,
                        mut_threshold=ga.rate_threshold(1, 2), nc=2, nr=3,
                        flags=ga.MUT_SHARED | ga.lanes_flag(lanes))
    _step_chain(cfg, 3)


def _run_gpu(cfg: ga.Config):
    pa, pb = empty_pop(cfg), empty_pop(cfg)
    ka, kb = empty_keys(cfg), empty_keys(cfg)
    res = ga.ga_run(cfg, pa, pb, ka, kb)
    final = pa if res["generation"] % 2 == 0 else pb
    fk = ka if res["generation"] % 2 == 0 else kb
    return res, int8_from_dev_pop(final, cfg.m), keys_np(fk)


def _same_run(cfg: ga.Config):
    res, pop, keys = _run_gpu(cfg)
    want, opop, okeys = gao.run(to_oracle(cfg))
    for k in ("found", "generation", "index", "best_key"):
        assert res[k] == want[k], (k, res, want)
    assert np.array_equal(res["matrix"], opop[want["index"]])
    assert np.array_equal(pop, opop) and np.array_equal(keys, okeys)
    return res


def test_run_plain_m8_config():
    """Plain GA, m=8, population 1024, seed 0, SQ, binary tournament,
    crossover 0.5, one pair flip at rate 0.1, 200 generations, stop at 0."""
    torch_cuda()
    announce("run m8 n1024")
    cfg = ga.Config(m=8, n=1024, seed=0, max_generations=200)
    res = _same_run(cfg)
    assert res["found"] and hf.is_hadamard(res["matrix"])


@pytest.mark.parametrize("cfg", [
    ga.Config(m=12, n=600, seed=3, max_generations=40, flags=0),
    ga.Config(m=4, n=64, seed=1, max_generations=50),
    ga.Config(m=16, n=2000, seed=5, elite=20, fitness=ga.FIT_SQ_PLUS_NNZ, max_generations=30),
    ga.Config(m=12, n=400, seed=8, selection=ga.SEL_PAPER, fitness=ga.FIT_F2,
              xo_threshold=1 << 32, mut_threshold=1 << 32, nc=1, nr=2, max_generations=300),
    ga.Config(m=36, n=300, seed=9, max_generations=6, flags=0),
    ga.Config(m=8, n=100, seed=0, max_generations=0),
    ga.Config(m=100, n=1000, seed=9100, selection=ga.SEL_PAPER, fitness=ga.FIT_F2,
              xo_threshold=1 << 32, mut_threshold=1 << 32, nc=4, nr=2, max_generations=12,
              flags=0),
    ga.Config(m=128, n=300, seed=12, max_generations=8, flags=0),
    ga.Config(m=84, n=500, seed=13, elite=10, fitness=ga.FIT_ABS, max_generations=10),
    ga.Config(m=12, n=400, seed=14, selection=ga.SEL_PAPER, fitness=ga.FIT_F2,
              xo_threshold=1 << 32, mut_threshold=1 << 32, nc=1, nr=1, max_generations=300,
              flags=ga.STOP_ON_FOUND | ga.MUT_SHARED),
    ga.Config(m=52, n=2000, seed=18, selection=ga.SEL_PAPER, fitness=ga.FIT_F1,
              xo_threshold=1 << 32, mut_threshold=1 << 32, nc=2, nr=3, max_generations=70,
              flags=0),
    # the one-block paper selection at its largest population (64 keys per
    # thread), and just past it (the multi-launch selection with a slot table)
    ga.Config(m=16, n=65536, seed=19, selection=ga.SEL_PAPER, fitness=ga.FIT_F2,
              xo_threshold=1 << 32, mut_threshold=1 << 32, nc=1, nr=2, max_generations=40,
              flags=0),
    ga.Config(m=8, n=65540, seed=20, selection=ga.SEL_PAPER, fitness=ga.FIT_F1,
              xo_threshold=1 << 32, mut_threshold=1 << 32, nc=1, nr=2, max_generations=10,
              flags=0),
    # the same, long enough for the run to measure its lanes per child on its
    # first generations (their selections reading the slot table's rows)
    ga.Config(m=8, n=65540, seed=21, selection=ga.SEL_PAPER, fitness=ga.FIT_F1,
              xo_threshold=1 << 32, mut_threshold=1 << 32, nc=1, nr=2, max_generations=200,
              flags=0),
    # the Table 2 configuration at m = 20 (40,000 matrices, F2, NC = 4, NR = 2),
    # shortened to 300 generations
    ga.Config(m=20, n=40000, seed=9020, selection=ga.SEL_PAPER, fitness=ga.FIT_F2,
              xo_threshold=1 << 32, mut_threshold=1 << 32, nc=4, nr=2, max_generations=300,
              flags=0),
    # 64 x 2N > 2^24: no chunk slot table, the scatter walks the permutation
    ga.Config(m=4, n=600000, seed=17, selection=ga.SEL_PAPER, fitness=ga.FIT_F2,
              xo_threshold=1 << 32, mut_threshold=1 << 32, nc=1, nr=1, max_generations=3,
              flags=0),
])
def test_run_parity(cfg):
    torch_cuda()
    announce("run", cfg)
    _same_run(cfg)


@pytest.mark.parametrize("cfg", [
    # keys 0, 16 and 48 only: ties everywhere, the elites' threshold among them
    ga.Config(m=4, n=1000, seed=1, elite=300, max_generations=40, flags=0),
    # almost every slot an elite: five child pairs, more elites than blocks
    ga.Config(m=8, n=600, seed=2, elite=590, max_generations=30, flags=0),
    ga.Config(m=12, n=5000, seed=3, elite=1, fitness=ga.FIT_NNZ, max_generations=100),
    ga.Config(m=20, n=3001, seed=4, elite=700, fitness=ga.FIT_ABS, max_generations=70, flags=0),
    ga.Config(m=32, n=20000, seed=5, elite=200, fitness=ga.FIT_SQ_PLUS_NNZ, max_generations=70,
              flags=0),
    ga.Config(m=44, n=2000, seed=6, elite=31, fitness=ga.FIT_F1, max_generations=66, flags=0),
    ga.Config(m=68, n=900, seed=7, elite=90, fitness=ga.FIT_F2, max_generations=20, flags=0),
    ga.Config(m=100, n=500, seed=8, elite=65, fitness=ga.FIT_ABS, max_generations=10, flags=0),
    # more items than the selection holds in LDS (10,240): its lists and bitmap in global memory
    ga.Config(m=12, n=30000, seed=9, elite=10000, fitness=ga.FIT_ABS, max_generations=12, flags=0),
    # more slots than its LDS bitmap covers (262,144)
    ga.Config(m=8, n=300000, seed=10, elite=50, max_generations=8, flags=0),
    # half the population elite, 8-way tournaments at m = 72: in generation 1
    # the threshold lies 4624 below the largest elite key, under the
    # selection's 4096-wide window (checked with the oracle)
    ga.Config(m=72, n=800, seed=11, elite=400, tournament_k=8, max_generations=6, flags=0),
])
def test_run_elitism(cfg):
    """Whole elitist runs through ga_run, whose elites come from the previous
    elites and the children below their largest key: equal to the oracle's
    runs, which rank the whole population."""
    torch_cuda()
    announce("run elitism", cfg)
    _same_run(cfg)


@pytest.mark.parametrize("m,nc,nr,kind,gens", [
    (12, 1, 1, ga.FIT_F1, 400), (12, 4, 4, ga.FIT_F2, 150), (16, 1, 4, ga.FIT_F2, 150),
    (16, 3, 2, ga.FIT_F1, 100),
])
def test_run_paper_study_cells(m, nc, nr, kind, gens):
    """Whole runs in the configuration of the mutation study of Sec. 4.3
    (n = 4000, crossover and mutation on every offspring), with the study's
    first seed per order and a shortened budget."""
    torch_cuda()
    announce("run paper study cell", m, nc, nr, kind)
    cfg = ga.Config(m=m, n=4000, seed=8_000_000 + 1000 * m, selection=ga.SEL_PAPER, fitness=kind,
                    xo_threshold=1 << 32, mut_threshold=1 << 32, nc=nc, nr=nr, max_generations=gens)
    _same_run(cfg)


@pytest.mark.parametrize("cfg", [
    ga.Config(m=20, n=1500, seed=31, max_generations=400, flags=0),
    ga.Config(m=40, n=400, seed=32, elite=5, fitness=ga.FIT_ABS, max_generations=300, flags=0),
    ga.Config(m=20, n=1500, seed=33, max_generations=700, flags=0),
    ga.Config(m=40, n=400, seed=34, elite=5, fitness=ga.FIT_ABS, max_generations=450, flags=0),
    # paper mode: the measured generations select and read the slot table as the chunks do
    ga.Config(m=16, n=2000, seed=35, selection=ga.SEL_PAPER, fitness=ga.FIT_F1,
              xo_threshold=1 << 32, mut_threshold=1 << 32, nc=2, nr=2, max_generations=650,
              flags=0),
    # m = 8 runs find a solution in about 14 generations: inside the measured ones
    ga.Config(m=8, n=1024, seed=36, max_generations=700),
    ga.Config(m=8, n=1024, seed=38, max_generations=700),
    # the shortest run that measures (four chunks)
    ga.Config(m=12, n=600, seed=37, elite=3, fitness=ga.FIT_NNZ, max_generations=193, flags=0),
])
def test_run_tunes_lanes_inside_the_run(cfg):
    """A run long enough to time every lanes-per-child variant on its own
    first generations (launched one by one, the variants in turn), then one
    that reuses the measured choice: both equal the oracle's run, and the
    choice is one of the variants."""
    torch_cuda()
    announce("run tuned twice", cfg)
    _same_run(cfg)
    lanes = ga.ga_tuned_lanes(cfg)
    assert lanes in ((2, 4, 8) if cfg.m <= 32 else (4, 8) if cfg.m <= 64 else (8, 16)), lanes
    _same_run(cfg)
    assert ga.ga_tuned_lanes(cfg) == lanes


# --------------------------------------------------------------------------
# Batched runs and the server
# --------------------------------------------------------------------------
def _mixed_configs():
    rng = np.random.default_rng(4)
    out = []
    for i in range(7):
        m = int(rng.choice([8, 12, 16, 20, 36, 44]))
        n = int(rng.integers(100, 1500))
        out.append(ga.Config(m=m, n=n, seed=4_000_000 + i, max_generations=int(rng.integers(5, 40)),
                             fitness=int(rng.choice([ga.FIT_SQ, ga.FIT_ABS, ga.FIT_NNZ]))))
    out.append(ga.Config(m=8, n=256, seed=1, max_generations=100))  # solves early
    out.append(ga.Config(m=96, n=300, seed=4_000_100, max_generations=6, fitness=ga.FIT_ABS))
    return out


def test_run_batch_equals_single_runs():
    torch_cuda()
    cfgs = _mixed_configs()
    announce("batch", len(cfgs))
    batch = ga.ga_run_batch(cfgs)
    for cfg, got in zip(cfgs, batch):
        want, opop, _ = gao.run(to_oracle(cfg))
        for k in ("found", "generation", "index", "best_key"):
            assert got[k] == want[k], (cfg, got, want)
        assert np.array_equal(got["matrix"], opop[want["index"]])


def _selecting_configs():
    """Runs that select every generation (paper mode, elitism) mixed with
    plain tournaments, three of them sharing order 12's launch."""
    paper = dict(selection=ga.SEL_PAPER, xo_threshold=1 << 32, mut_threshold=1 << 32)
    return [
        ga.Config(m=12, n=400, seed=61, fitness=ga.FIT_F2, nc=1, nr=2, max_generations=40, **paper),
        ga.Config(m=12, n=301, seed=62, max_generations=25),
        ga.Config(m=12, n=500, seed=63, elite=9, fitness=ga.FIT_NNZ, max_generations=20, flags=0),
        ga.Config(m=20, n=700, seed=64, elite=7, fitness=ga.FIT_SQ, max_generations=12, flags=0),
        ga.Config(m=36, n=240, seed=65, fitness=ga.FIT_F1, nc=3, nr=2, max_generations=8, flags=0,
                  **paper),
        ga.Config(m=68, n=120, seed=66, fitness=ga.FIT_F2, nc=2, nr=2, max_generations=5, flags=0,
                  **paper),
        ga.Config(m=8, n=256, seed=67, fitness=ga.FIT_F2, nc=1, nr=1, max_generations=200,
                  flags=ga.STOP_ON_FOUND | ga.MUT_SHARED, **paper),
        ga.Config(m=16, n=4000, seed=68, fitness=ga.FIT_F2, nc=2, nr=2, max_generations=45,
                  flags=0, **paper),
    ]


def _equals_oracle_run(cfg, got):
    want, opop, _ = gao.run(to_oracle(cfg))
    for k in ("found", "generation", "index", "best_key"):
        assert got[k] == want[k], (cfg, got, want)
    assert np.array_equal(got["matrix"], opop[want["index"]])


def test_run_batch_with_selection():
    """Batched runs with paper-mode and elitist selection (each run's own
    selection launches before its order's shared children launch) equal
    their single runs in the oracle."""
    torch_cuda()
    cfgs = _selecting_configs()
    announce("batch with selection", len(cfgs))
    for cfg, got in zip(cfgs, ga.ga_run_batch(cfgs)):
        _equals_oracle_run(cfg, got)


def test_run_batch_paper_runs_share_selection_launches():
    """Several paper-mode runs of one order, of one to three selection tiles
    (4,096 keys each) and different kinds and flags, select in the same two
    launches per generation: each equals its run in the oracle."""
    torch_cuda()
    paper = dict(selection=ga.SEL_PAPER, xo_threshold=1 << 32, mut_threshold=1 << 32)
    cfgs = [
        ga.Config(m=12, n=8200, seed=71, fitness=ga.FIT_F2, nc=1, nr=2, max_generations=60,
                  flags=0, **paper),
        ga.Config(m=12, n=4096, seed=72, fitness=ga.FIT_F1, nc=2, nr=1, max_generations=45,
                  flags=0, **paper),
        ga.Config(m=12, n=400, seed=73, fitness=ga.FIT_F2, nc=1, nr=1, max_generations=200,
                  flags=ga.STOP_ON_FOUND, **paper),
        ga.Config(m=12, n=12000, seed=74, fitness=ga.FIT_SQ, nc=3, nr=2, max_generations=33,
                  flags=ga.MUT_SHARED, **paper),
        ga.Config(m=12, n=900, seed=75, max_generations=30),
    ]
    announce("batch paper runs sharing launches", len(cfgs))
    for cfg, got in zip(cfgs, ga.ga_run_batch(cfgs)):
        _equals_oracle_run(cfg, got)


def test_run_batch_elitist_runs_share_elite_launch():
    """Several elitist runs of one order choose their elites from candidate
    lists in one shared launch per generation (each block one run): ties
    (m = 4 keys take three values), almost every slot an elite, one elite,
    kinds with one- and two-level key ranges, a run whose items exceed the
    LDS; each equals the oracle's run."""
    torch_cuda()
    cfgs = [
        ga.Config(m=4, n=1000, seed=81, elite=300, max_generations=40, flags=0),
        ga.Config(m=4, n=600, seed=82, elite=590, fitness=ga.FIT_ABS, max_generations=30, flags=0),
        ga.Config(m=20, n=5000, seed=83, elite=1, fitness=ga.FIT_NNZ, max_generations=60),
        ga.Config(m=20, n=3001, seed=84, elite=700, fitness=ga.FIT_ABS, max_generations=50, flags=0),
        ga.Config(m=20, n=20000, seed=85, elite=200, fitness=ga.FIT_SQ_PLUS_NNZ, max_generations=40,
                  flags=0),
        # more items than the selection holds in LDS: its scratch in global memory
        ga.Config(m=20, n=24000, seed=88, elite=11000, fitness=ga.FIT_ABS, max_generations=10,
                  flags=0),
        ga.Config(m=20, n=900, seed=86, max_generations=30),
        ga.Config(m=20, n=800, seed=87, selection=ga.SEL_PAPER, fitness=ga.FIT_F2,
                  xo_threshold=1 << 32, mut_threshold=1 << 32, nc=2, nr=1, max_generations=35,
                  flags=0),
    ]
    announce("batch elitist runs sharing the elite launch", len(cfgs))
    for cfg, got in zip(cfgs, ga.ga_run_batch(cfgs)):
        _equals_oracle_run(cfg, got)


def test_server_with_selection():
    torch_cuda()
    cfgs = _selecting_configs()
    announce("server with selection", len(cfgs))
    srv = ga.Server(hbm_budget_bytes=1 << 30)
    try:
        ids = [srv.submit(c) for c in cfgs]
        for cfg, i in zip(cfgs, ids):
            _equals_oracle_run(cfg, srv.wait(i))
    finally:
        srv.close()


@pytest.mark.parametrize("lanes", ["tuned", "fewest", "most"])
def test_run_batch_every_order(lanes):
    """One run of every order 4..128 in one batched launch sequence: each
    order has its own batched children kernel, with the tuned, the fewest
    or the most lanes per child."""
    torch_cuda()
    kinds = [ga.FIT_SQ, ga.FIT_ABS, ga.FIT_NNZ, ga.FIT_SQ_PLUS_NNZ, ga.FIT_F1, ga.FIT_F2]

    def flags(m):
        if lanes == "tuned":
            return 0
        return ga.lanes_flag(lanes_of(m)[0] if lanes == "fewest" else lanes_of(m)[-1])
    cfgs = [ga.Config(m=m, n=200 + 37 * i, seed=7_000_000 + m, fitness=kinds[i % 6],
                      max_generations=4 + i % 5, flags=flags(m), nc=1 + i % 2, nr=1 + i % 3)
            for i, m in enumerate(ORDERS)]
    announce("batch every order", len(cfgs))
    batch = ga.ga_run_batch(cfgs)
    for cfg, got in zip(cfgs, batch):
        want, opop, _ = gao.run(to_oracle(cfg))
        for k in ("found", "generation", "index", "best_key"):
            assert got[k] == want[k], (cfg, got, want)
        assert np.array_equal(got["matrix"], opop[want["index"]])


def test_server_results_equal_alone_and_mixed():
    torch_cuda()
    cfgs = _mixed_configs()
    announce("server", len(cfgs))
    srv = ga.Server(hbm_budget_bytes=1 << 30)
    try:
        ids = [srv.submit(c) for c in cfgs]
        mixed = [srv.wait(i) for i in ids]
        alone = []
        for c in cfgs:
            alone.append(srv.wait(srv.submit(c)))
        for c, a, b in zip(cfgs, mixed, alone):
            want, opop, _ = gao.run(to_oracle(c))
            for k in ("found", "generation", "index", "best_key"):
                assert a[k] == b[k] == want[k]
            assert np.array_equal(a["matrix"], b["matrix"])
            assert np.array_equal(a["matrix"], opop[want["index"]])
        assert all(srv.latency(i) > 0 for i in ids)
    finally:
        srv.close()


def test_server_small_budget_queues():
    """A budget that holds only one request at a time still serves all of
    them, in order, and rejects a request that can never fit."""
    torch_cuda()
    cfg = ga.Config(m=20, n=2000, seed=3, max_generations=10, flags=0)
    one = 2 * (((2000 * 20 * 4) + 255) // 256 * 256) + 2 * (((2000 * 4) + 255) // 256 * 256)
    announce("server small budget", one)
    srv = ga.Server(hbm_budget_bytes=one + 100)
    try:
        ids = [srv.submit(ga.Config(**{**cfg.__dict__, "seed": s})) for s in range(4)]
        res = [srv.wait(i) for i in ids]
        for s, r in zip(range(4), res):
            want, _, _ = gao.run(to_oracle(ga.Config(**{**cfg.__dict__, "seed": s})))
            assert r["best_key"] == want["best_key"] and r["index"] == want["index"]
        big = ga.Config(m=20, n=4000, seed=1, max_generations=1)
        with pytest.raises(ga.GAError) as e:
            srv.submit(big)
        assert e.value.status == ga.GA_EBUDGET
    finally:
        srv.close()


# --------------------------------------------------------------------------
# The m=20, population 40,000 workload at full size
# --------------------------------------------------------------------------
def test_full_size_m20_n40000_generations():
    """Full-size check of the m=20, n=40,000 workload in the launch
    configuration the benchmark times: init, fitness (SQ and ABS keys with
    components) and the first generations, against the oracle."""
    torch = torch_cuda()
    for kind in (ga.FIT_SQ, ga.FIT_ABS):
        announce("full m20 n40000", kind)
        cfg = ga.Config(m=20, n=40000, seed=1, fitness=kind, max_generations=500, flags=0)
        ocfg = to_oracle(cfg)
        dpop, dkeys = empty_pop(cfg), empty_keys(cfg)
        comps = torch.zeros((cfg.n, 3), dtype=torch.int32, device="cuda")
        ga.ga_init_population(cfg, dpop)
        ga.ga_fitness(cfg, dpop, dkeys, comps)
        pop = gao.init_population(ocfg)
        keys, oc = gao.fitness(ocfg, pop, with_comps=True)
        assert np.array_equal(int8_from_dev_pop(dpop, 20), pop)
        assert np.array_equal(keys_np(dkeys), keys)
        assert np.array_equal(comps.cpu().numpy().view(np.uint32), oc)
        nxt, nk = empty_pop(cfg), empty_keys(cfg)
        for g in range(2):
            ga.ga_step(cfg, dpop, dkeys, nxt, nk, g)
            pop, keys = gao.step(ocfg, pop, keys, g)
            assert np.array_equal(keys_np(nk), keys)
            assert np.array_equal(int8_from_dev_pop(nxt, 20), pop)
            dpop, nxt, dkeys, nk = nxt, dpop, nk, dkeys


def test_full_size_m32_n200000_elite_generation():
    """The m=32, n=200,000 workload with 2,000 elites and key SQ+NNZ:
    one generation against the oracle."""
    torch_cuda()
    announce("full m32 n200000 elite")
    cfg = ga.Config(m=32, n=200000, seed=2, fitness=ga.FIT_SQ_PLUS_NNZ, elite=2000,
                    max_generations=1000, flags=0)
    ocfg = to_oracle(cfg)
    dpop, dkeys = empty_pop(cfg), empty_keys(cfg)
    ga.ga_init_population(cfg, dpop)
    ga.ga_fitness(cfg, dpop, dkeys)
    pop = gao.init_population(ocfg)
    keys = gao.fitness(ocfg, pop)
    assert np.array_equal(keys_np(dkeys), keys)
    nxt, nk = empty_pop(cfg), empty_keys(cfg)
    ga.ga_step(cfg, dpop, dkeys, nxt, nk, 0)
    pop, keys = gao.step(ocfg, pop, keys, 0)
    assert np.array_equal(keys_np(nk), keys)
    assert np.array_equal(int8_from_dev_pop(nxt, 32), pop)


def test_full_size_table2_m100_n40000_run():
    """The Table 2 configuration at its full size (m = 100, 40,000 matrices,
    paper mode, F2, NC = 4, NR = 2, the benchmark's seed) through ga_run,
    whose chunk computes the slot permutations in one launch: two whole
    generations, population and keys, against the oracle."""
    torch_cuda()
    announce("full table2 m100 n40000")
    cfg = ga.Config(m=100, n=40000, seed=9100, selection=ga.SEL_PAPER, fitness=ga.FIT_F2,
                    xo_threshold=1 << 32, mut_threshold=1 << 32, nc=4, nr=2,
                    max_generations=2, flags=0)
    _same_run(cfg)


def test_invalid_configs_rejected():
    torch_cuda()
    bad = ga.Config(m=18, n=100)
    pop = empty_pop(bad)
    with pytest.raises(ga.GAError) as e:
        ga.ga_init_population(bad, pop)
    assert e.value.status == ga.GA_EINVAL
    with pytest.raises(ga.GAError) as e:  # one invalid run rejects the batch
        ga.ga_run_batch([ga.Config(m=8, n=100, elite=2), ga.Config(m=18, n=100)])
    assert e.value.status == ga.GA_EINVAL


# --------------------------------------------------------------------------
# Whole runs of the benchmarked configurations, through the timed entry
# points (ga_run's captured chunks and in-run lane measurement, the batched
# launches, the server), against the oracle's whole runs
# --------------------------------------------------------------------------
import hashlib  # noqa: E402
import json  # noqa: E402
import os  # noqa: E402

GOLDEN_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _golden(name):
    """Stored oracle results, written by tests/golden/make_golden.py (which
    calls only the oracle)."""
    with open(os.path.join(GOLDEN_DIR, name)) as f:
        return json.load(f)


def _digest(a) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def _rows(Q) -> list:
    return ["".join("+" if x > 0 else "-" for x in row) for row in Q]


def _equals_record(got, rec):
    for k in ("found", "generation", "index", "best_key"):
        assert got[k] == rec[k], (k, got[k], rec[k], rec["config"])
    assert _rows(got["matrix"]) == rec["matrix"], rec["config"]


def _from_fields(f) -> ga.Config:
    f = dict(f)
    stop = f.pop("stop_on_found")
    return ga.Config(**f, flags=ga.STOP_ON_FOUND if stop else 0)


@pytest.mark.parametrize("kind", [ga.FIT_SQ, ga.FIT_ABS])
def test_full_size_m20_n40000_whole_run(kind):
    """The benchmark's timed path at full size: ga_run at m = 20, n = 40,000,
    seed 1, 500 generations, no stop on found, SQ and ABS keys.  The first
    call measures the lanes per child on its own first generations, the
    second reuses the measured choice (as the timed benchmark steps do);
    both leave the oracle's final population and keys and report its
    result."""
    torch_cuda()
    cfg = ga.Config(m=20, n=40000, seed=1, fitness=kind, max_generations=500, flags=0)
    announce("whole run m20 n40000", kind)
    want, opop, okeys = gao.run(to_oracle(cfg))
    for call in range(2):
        res, pop, keys = _run_gpu(cfg)
        for k in ("found", "generation", "index", "best_key"):
            assert res[k] == want[k], (call, k, res, want)
        assert np.array_equal(res["matrix"], opop[want["index"]])
        assert np.array_equal(keys, okeys), call
        assert np.array_equal(pop, opop), call


def test_full_size_m32_n200000_elite_20_generations():
    """The elitist configuration (m = 32, n = 200,000, seed 2, SQ + NNZ,
    2,000 elites) through ga_run for 20 generations: final population, keys
    and result equal the oracle's run."""
    torch_cuda()
    announce("whole run m32 n200000 elite, 20 generations")
    _same_run(ga.Config(m=32, n=200000, seed=2, fitness=ga.FIT_SQ_PLUS_NNZ, elite=2000,
                        max_generations=20, flags=0))


def test_full_size_m32_n200000_elite_1000_generations():
    """The same configuration over its whole 1,000-generation budget (the
    benchmark's elitist run), twice (lane measurement, then the measured
    choice): result and digests of the final population and keys equal the
    stored oracle run."""
    torch_cuda()
    rec = _golden("elite_m32_n200000.json")["run"]
    cfg = _from_fields(rec["config"])
    assert (cfg.m, cfg.n, cfg.elite, cfg.max_generations) == (32, 200000, 2000, 1000)
    for call in range(2):
        announce("whole run m32 n200000 elite, 1000 generations", call)
        res, pop, keys = _run_gpu(cfg)
        _equals_record(res, rec)
        assert _digest(keys.astype("<u4")) == rec["keys_sha256"], call
        assert _digest(pop) == rec["population_sha256"], call


@pytest.mark.parametrize("key", ["F1", "F2"])
def test_full_size_table2_m20_paper_mode_10000_generations(key):
    """The benchmark's paper-mode leg at full size (Sec. 4.2 timing
    configuration at m = 20: 40,000 matrices, NC = 4, NR = 2, 10^4
    generations, no stop on found), twice (lane measurement, then the
    measured choice): result and digests of the final population and keys
    equal the stored oracle run."""
    torch_cuda()
    runs = _golden("paper_table2_m20.json")["runs"]
    rec = runs[0 if key == "F1" else 1]
    cfg = _from_fields(rec["config"])
    assert (cfg.m, cfg.n, cfg.max_generations, cfg.nc, cfg.nr) == (20, 40000, 10000, 4, 2)
    assert cfg.fitness == (ga.FIT_F1 if key == "F1" else ga.FIT_F2)
    for call in range(2):
        announce("whole run table2 m20", key, call)
        res, pop, keys = _run_gpu(cfg)
        _equals_record(res, rec)
        assert _digest(keys.astype("<u4")) == rec["keys_sha256"], call
        assert _digest(pop) == rec["population_sha256"], call


def test_batched_workload_24_runs_equal_oracle():
    """The batched benchmark workload at full size (24 runs, orders 12..36,
    populations 2,000..60,000, 300 generations): every run of the batched
    launches reports the stored oracle run's result, and each run alone
    through ga_run leaves the oracle's final population and keys."""
    torch_cuda()
    recs = _golden("batched_24runs.json")["runs"]
    cfgs = [_from_fields(f) for f in inputs.batched_workload()]
    assert [r["config"] for r in recs] == inputs.batched_workload()
    announce("batched workload", len(cfgs))
    for got, rec in zip(ga.ga_run_batch(cfgs), recs):
        _equals_record(got, rec)
    for cfg, rec in zip(cfgs, recs):
        announce("batched workload run alone", cfg.m, cfg.n, cfg.seed)
        res, pop, keys = _run_gpu(cfg)
        _equals_record(res, rec)
        assert _digest(keys.astype("<u4")) == rec["keys_sha256"]
        assert _digest(pop) == rec["population_sha256"]


def test_served_stream_slice_equals_plain_runs_and_oracle():
    """The first 200 requests of the served benchmark's stream (orders 8..64,
    populations 1,000..50,000, 2,000-generation budget, stop on found), all
    submitted to one server: each result equals the same request's ga_run,
    and the requests of order <= 16 equal the stored oracle runs."""
    torch_cuda()
    gold = _golden("served_slice.json")
    fields, _ = inputs.served_workload()
    cfgs = [_from_fields(f) for f in fields[:gold["requests"]]]
    announce("served slice", len(cfgs))
    srv = ga.Server(hbm_budget_bytes=200 * 10**9)
    try:
        ids = [srv.submit(c) for c in cfgs]
        served = [srv.wait(i) for i in ids]
    finally:
        srv.close()
    by_request = {r["request"]: r for r in gold["runs"]}
    assert sorted(by_request) == [i for i, c in enumerate(cfgs) if c.m <= gold["max_order"]]
    for i, rec in by_request.items():
        assert rec["config"] == fields[i]
        _equals_record(served[i], rec)
    cache = {}
    for i, (cfg, got) in enumerate(zip(cfgs, served)):
        shape = (cfg.m, cfg.n)
        if shape not in cache:
            cache.clear()
            cache[shape] = (empty_pop(cfg), empty_pop(cfg), empty_keys(cfg), empty_keys(cfg))
        want = ga.ga_run(cfg, *cache[shape])
        for k in ("found", "generation", "index", "best_key"):
            assert got[k] == want[k], (i, k, got[k], want[k])
        assert np.array_equal(got["matrix"], want["matrix"]), i


def _run_bytes(cfg: ga.Config) -> int:
    """Device bytes of a tournament run without elites on the server: two
    populations and two key arrays, each rounded up to 256 bytes."""
    pop = cfg.n * cfg.m * cfg.words * 4
    return 2 * ((pop + 255) // 256 * 256) + 2 * ((cfg.n * 4 + 255) // 256 * 256)


def test_server_small_request_passes_a_waiting_large_one():
    """A request that does not fit the budget beside a running one waits,
    while a later small request that fits is admitted and finishes first;
    the large one runs once memory frees up.  Every result equals the
    oracle's."""
    torch_cuda()
    long_run = ga.Config(m=8, n=2000, seed=21, max_generations=2000, flags=0)
    large = ga.Config(m=8, n=2200, seed=22, max_generations=5, flags=0)
    small = ga.Config(m=8, n=200, seed=23, max_generations=5, flags=0)
    budget = max(_run_bytes(large), _run_bytes(long_run) + _run_bytes(small)) + 1024
    assert _run_bytes(large) + _run_bytes(long_run) > budget
    announce("server bypass", budget)
    srv = ga.Server(hbm_budget_bytes=budget)
    try:
        ids = [srv.submit(c) for c in (long_run, large, small)]
        res = [srv.wait(i) for i in ids]
        lat = [srv.latency(i) for i in ids]
    finally:
        srv.close()
    assert lat[2] < lat[0] < lat[1], lat
    for cfg, got in zip((long_run, large, small), res):
        _equals_oracle_run(cfg, got)


def test_server_stop_fails_unfinished_and_refuses_submissions():
    """ga_server_stop ends the worker: a finished result stays readable, the
    requests still queued or running fail with GA_ESTOPPED, and a later
    submission is refused with the same status."""
    torch_cuda()
    quick = ga.Config(m=8, n=256, seed=1, max_generations=100)
    slow = ga.Config(m=36, n=20000, seed=5, max_generations=1_000_000, flags=0)
    announce("server stop")
    srv = ga.Server(hbm_budget_bytes=1 << 30)
    try:
        q = srv.submit(quick)
        done = srv.wait(q)
        ids = [srv.submit(ga.Config(**{**slow.__dict__, "seed": s})) for s in range(3)]
        srv.stop()
        for i in ids:
            with pytest.raises(ga.GAError) as e:
                srv.wait(i)
            assert e.value.status == ga.GA_ESTOPPED
        with pytest.raises(ga.GAError) as e:
            srv.submit(quick)
        assert e.value.status == ga.GA_ESTOPPED
        assert srv.wait(q)["best_key"] == done["best_key"]
        _equals_oracle_run(quick, done)
    finally:
        srv.close()
