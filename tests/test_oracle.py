"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: published
Philox known-answer vectors, textbook Hadamard constructions, an exhaustive
census at m=4 derived by hand, closed forms, the paper's two worked figures,
and distributional facts of the operators.
"""
import itertools
import json
import math
import os

import numpy as np
import pytest
from scipy import stats

from oracle import gao
from tests import hadamard_fixtures as hf
from tests import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _mat(rows):
    return np.array([[1 if ch == "+" else -1 for ch in r] for r in rows], dtype=np.int8)


# --------------------------------------------------------------------------
# Philox4x32-10 and the draw helpers
# --------------------------------------------------------------------------
# Known-answer vectors of Philox4x32-10 published with the Random123 library
# that accompanies Salmon et al. (SC'11): (counter, key) -> output.
PHILOX_KAT = [
    ([0, 0, 0, 0], [0, 0], [0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8]),
    ([0xFFFFFFFF] * 4, [0xFFFFFFFF] * 2, [0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD]),
    ([0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344], [0xA4093822, 0x299F31D0],
     [0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1]),
]


@pytest.mark.parametrize("ctr,key,want", PHILOX_KAT)
def test_philox_known_answers(ctr, key, want):
    assert list(gao.philox(ctr, key)) == want


def test_draw_counter_layout():
    seed = (7 << 32) | 123456789
    for (stream, gen, idx, d) in [(1, 0, 0, 0), (2, 5, 17, 3), (4, 1 << 20, 99, 13)]:
        block = gao.philox([d // 4, idx, gen, stream], [seed & 0xFFFFFFFF, seed >> 32])
        assert gao.draw(seed, stream, gen, idx, d) == block[d % 4]


def test_bounded_edges():
    for r in [1, 2, 3, 19, 40000, 2**31 + 5]:
        assert gao.bounded(0, r) == 0
        assert gao.bounded(0xFFFFFFFF, r) == r - 1
        assert gao.bounded(1 << 31, r) == r // 2
    # the mapping is monotone and hits every value of a small range equally
    hits = np.bincount([gao.bounded(u << 24, 7) for u in range(256)], minlength=7)
    assert hits.min() >= 36 and hits.max() <= 37


def test_draws_uniform():
    u = np.array([gao.draw(3, 2, g, i, d) for g in range(4) for i in range(64)
                  for d in range(16)], dtype=np.uint64)
    counts = np.bincount((u >> np.uint64(28)).astype(np.int64), minlength=16)
    assert stats.chisquare(counts).pvalue > 1e-4


# --------------------------------------------------------------------------
# Gram matrix and fitness
# --------------------------------------------------------------------------
@pytest.mark.parametrize("m", hf.ORDERS_WITH_FIXTURE)
def test_known_hadamard_has_zero_fitness(m):
    H = hf.hadamard(m)
    G = gao.gram(H)
    assert np.array_equal(G, m * np.eye(m, dtype=np.int32))
    for kind in range(6):
        key, comps = gao.fitness_one(H, kind)
        assert key == 0 and comps == (0, 0, 0)


def test_m4_census():
    """All 216 normalized 4x4 matrices with balanced columns.

    Two balanced +-1 columns of length 4 have dot product 4 (equal), -4
    (complementary) or 0.  The 6 balanced columns form 3 complementary
    pairs, so three columns are mutually orthogonal iff they come from 3
    different pairs: 3! * 2^3 = 48 matrices.  Exactly one non-orthogonal
    column pair: 3 (which pair) * 3 (its class) * 4 (signs) * 4 (third
    column) = 144.  All three from one class: 3 * 2^3 = 24.
    """
    pops = inputs.all_m4_normalized()
    seen = {}
    for Q in pops:
        key, comps = gao.fitness_one(Q, gao.FIT_SQ)
        seen[comps] = seen.get(comps, 0) + 1
        assert gao.fitness_one(Q, gao.FIT_F1)[0] == 2 * comps[1]
        assert gao.fitness_one(Q, gao.FIT_F2)[0] == 2 * comps[2]
        assert gao.fitness_one(Q, gao.FIT_SQ_PLUS_NNZ)[0] == comps[0] + comps[2]
    assert seen == {(0, 0, 0): 48, (16, 4, 1): 144, (48, 12, 3): 24}


@pytest.mark.parametrize("m", [4, 8, 20, 32, 36, 64, 68, 100, 128])
def test_all_equal_columns_closed_form(m):
    """Columns 1..m-1 identical and balanced: every pair has dot product m."""
    Q = np.ones((m, m), dtype=np.int8)
    Q[: m // 2, 1:] = -1
    P = (m - 1) * (m - 2) // 2
    key, comps = gao.fitness_one(Q, gao.FIT_SQ)
    assert comps == (P * m * m, P * m, P)
    assert gao.fitness_one(Q, gao.FIT_F1)[0] == 2 * P * m
    assert gao.fitness_one(Q, gao.FIT_F2)[0] == 2 * P


@pytest.mark.parametrize("m", [8, 12, 20, 28, 32, 44, 64, 72, 100, 128])
def test_fitness_matches_row_space_identity(m):
    """sum_ij (Q^T Q)_ij^2 = sum_rs (Q Q^T)_rs^2 (Frobenius norms agree), so
    SQ = (||Q Q^T||_F^2 - m * m^2) / 2 is computed here from rows only; ABS
    and NNZ are checked against numpy's Gram product."""
    pop = inputs.random_population(m, 24, seed=m)
    cfg = gao.Config(m=m, n=24)
    keys, comps = gao.fitness(cfg, pop, with_comps=True)
    for Q, k, (sq, ab, nz) in zip(pop, keys, comps):
        R = Q.astype(np.int64) @ Q.astype(np.int64).T
        assert sq == ((R * R).sum() - m ** 3) // 2
        G = Q.astype(np.int64).T @ Q.astype(np.int64)
        iu = np.triu_indices(m, 1)
        assert ab == np.abs(G[iu]).sum() and nz == np.count_nonzero(G[iu])
        assert k == sq
        # balanced columns: every dot product is 0 mod 4
        assert sq % 16 == 0 and ab % 4 == 0


# --------------------------------------------------------------------------
# Initial population
# --------------------------------------------------------------------------
@pytest.mark.parametrize("m,n", [(4, 500), (8, 200), (20, 50), (64, 10), (100, 6), (128, 4)])
def test_init_invariants_and_determinism(m, n):
    cfg = gao.Config(m=m, n=n, seed=11)
    pop = gao.init_population(cfg)
    assert gao.check_invariants(pop) == 0
    assert np.array_equal(pop, gao.init_population(cfg))
    other = gao.init_population(gao.Config(m=m, n=n, seed=12))
    assert not np.array_equal(pop, other)


def test_init_column_patterns_uniform_m4():
    """Each column 1..3 is uniform over the 6 balanced patterns, and all 216
    matrices appear (a shuffle bug skews or misses patterns)."""
    n = 6000
    pop = gao.init_population(gao.Config(m=4, n=n, seed=5))
    code = ((pop == -1).astype(np.int64) * (1 << np.arange(4))[None, :, None]).sum(axis=1)
    balanced = [c for c in range(16) if bin(c).count("1") == 2]
    for j in (1, 2, 3):
        counts = np.array([np.count_nonzero(code[:, j] == c) for c in balanced])
        assert counts.sum() == n
        assert stats.chisquare(counts).pvalue > 1e-4
    whole = {tuple(r) for r in code[:, 1:]}
    assert len(whole) == 216


def test_init_m8_first_row_frequency():
    """For m=8 each entry of columns 1..7 is -1 with probability 1/2."""
    pop = gao.init_population(gao.Config(m=8, n=4000, seed=9))
    frac = (pop[:, :, 1:] == -1).mean(axis=0)
    assert np.abs(frac - 0.5).max() < 0.04


# --------------------------------------------------------------------------
# Crossover and mutation: the paper's figures
# --------------------------------------------------------------------------
def test_crossover_figure():
    fx = json.load(open(os.path.join(GOLDEN, "crossover_figure.json")))
    O0, O1 = gao.crossover(_mat(fx["P1"]), _mat(fx["PN1"]), fx["cut"])
    assert np.array_equal(O0, _mat(fx["O1"]))
    assert np.array_equal(O1, _mat(fx["ON1"]))


def test_crossover_exhaustive_m4():
    pops = inputs.all_m4_normalized()
    rng = np.random.default_rng(0)
    for a, b in rng.integers(0, len(pops), size=(300, 2)):
        A, B = pops[a], pops[b]
        for cut in (1, 2, 3):
            O0, O1 = gao.crossover(A, B, cut)
            for j in range(4):
                src0, src1 = (A, B) if j < cut else (B, A)
                assert np.array_equal(O0[:, j], src0[:, j])
                assert np.array_equal(O1[:, j], src1[:, j])
            assert gao.check_invariants(np.stack([O0, O1])) == 0


@pytest.mark.parametrize("panel", ["a", "b", "c", "d"])
def test_mutation_figure(panel):
    fx = json.load(open(os.path.join(GOLDEN, "mutation_figure.json")))["panels"][panel]
    r1 = fx.get("rowindx1_read", fx["rowindx1"])
    r2 = fx.get("rowindx2_read", fx["rowindx2"])
    Q = _mat(fx["matrix"])
    out = gao.mutate(Q, fx["colindx"], r1, r2)
    changed = {(int(i), int(j)) for i, j in zip(*np.nonzero(out != Q))}
    flipped = {tuple(c) for c in fx["colours"]["green"] + fx["colours"]["blue"]}
    kept = {tuple(c) for c in fx["colours"]["red"] + fx["colours"]["magenta"]}
    assert changed == flipped
    assert not (changed & kept)
    assert gao.check_invariants(out[None]) == 0


def test_mutation_panel_a_printed_indices_disagree():
    """The indices printed for panel (a) do not reproduce its colours."""
    fx = json.load(open(os.path.join(GOLDEN, "mutation_figure.json")))["panels"]["a"]
    Q = _mat(fx["matrix"])
    out = gao.mutate(Q, fx["colindx"], fx["rowindx1"], fx["rowindx2"])
    changed = {(int(i), int(j)) for i, j in zip(*np.nonzero(out != Q))}
    flipped = {tuple(c) for c in fx["colours"]["green"] + fx["colours"]["blue"]}
    assert changed != flipped


def test_mutation_sequential_semantics():
    Q = inputs.random_population(8, 1, seed=3)[0]
    col = 3
    rows = np.nonzero(Q[:, col] == -1)[0]
    other = np.nonzero(Q[:, col] == 1)[0]
    r1, r2 = int(rows[0]), int(other[0])
    once = gao.mutate(Q, [col], [r1], [r2])
    assert once[r1, col] == 1 and once[r2, col] == -1
    assert np.array_equal(gao.mutate(Q, [col], [r1, r1], [r2, r2]), Q)  # flips back
    assert np.array_equal(gao.mutate(Q, [col], [r1], [r1]), Q)          # same row: no-op
    same = int(rows[1])
    assert np.array_equal(gao.mutate(Q, [col], [r1], [same]), Q)        # equal signs


# --------------------------------------------------------------------------
# Selection helpers
# --------------------------------------------------------------------------
def test_select_set_matches_lexsort():
    rng = np.random.default_rng(1)
    keys = rng.integers(0, 30, size=1000).astype(np.uint32)
    for count in (1, 10, 500, 999, 1000):
        want = np.sort(np.lexsort((np.arange(1000), keys))[:count])
        assert np.array_equal(gao.select_set(keys, count), want)


@pytest.mark.parametrize("domain", [2, 3, 5, 16, 17, 100, 1000, 4097])
def test_permute_is_a_permutation(domain):
    img = [gao.permute(42, 7, domain, s) for s in range(domain)]
    assert sorted(img) == list(range(domain))


def test_permute_position_distribution():
    D, trials = 10, 3000
    counts = np.zeros((D, D), dtype=np.int64)
    for g in range(trials):
        for s in range(D):
            counts[s, gao.permute(5, g, D, s)] += 1
    assert stats.chisquare(counts.ravel()).pvalue > 1e-4


def test_permute_pair_distribution():
    """The ordered pair (pi(0), pi(1)) is uniform over the D(D-1) pairs."""
    D, trials = 6, 6000
    counts = np.zeros((D, D), dtype=np.int64)
    for g in range(trials):
        counts[gao.permute(9, g, D, 0), gao.permute(9, g, D, 1)] += 1
    assert np.trace(counts) == 0
    off = counts[~np.eye(D, dtype=bool)]
    assert stats.chisquare(off).pvalue > 1e-4


def test_tournament_winner_distribution():
    """Binary tournament with replacement over distinct keys: the winner has
    rank r (0 = best) with probability ((n-r)^2 - (n-r-1)^2) / n^2."""
    n = 20
    keys = np.random.default_rng(4).permutation(n).astype(np.uint32)
    rank = np.argsort(np.argsort(keys))
    cfg = gao.Config(m=8, n=n, seed=17, tournament_k=2)
    counts = np.zeros(n, dtype=np.int64)
    for p in range(6000):
        a, b = gao.tournament_parents(cfg, keys, 3, p)
        counts[rank[a]] += 1
        counts[rank[b]] += 1
    r = np.arange(n)
    prob = ((n - r) ** 2 - (n - r - 1) ** 2) / n ** 2
    assert stats.chisquare(counts, prob * counts.sum()).pvalue > 1e-4


def test_tournament_ties_go_to_lower_index():
    keys = np.zeros(50, dtype=np.uint32)
    cfg = gao.Config(m=8, n=50, seed=2, tournament_k=3)
    for p in range(200):
        a, _ = gao.tournament_parents(cfg, keys, 1, p)
        xs = [gao.bounded(gao.draw(2, gao.STREAM_SELECT, 1, p, k), 50) for k in range(3)]
        assert a == min(xs)


# --------------------------------------------------------------------------
# Whole generations
# --------------------------------------------------------------------------
def _children_consistent(cfg, pop, keys, pop2, keys2, gen_in):
    """Every child is a column mix of its two tournament parents, differing
    from the pure crossover in at most nc columns, with its fitness key."""
    e = cfg.elite
    for p in range((cfg.n - e + 1) // 2):
        a, b = gao.tournament_parents(cfg, keys, gen_in + 1, p)
        for ch in range(2):
            s = e + 2 * p + ch
            if s >= cfg.n:
                continue
            C = pop2[s]
            bad = 0
            for j in range(cfg.m):
                if not (np.array_equal(C[:, j], pop[a][:, j]) or np.array_equal(C[:, j], pop[b][:, j])):
                    bad += 1
            assert bad <= cfg.nc
            assert keys2[s] == gao.fitness_one(C, cfg.fitness)[0]


@pytest.mark.parametrize("m,n,elite", [(8, 64, 0), (12, 51, 0), (20, 40, 4), (36, 17, 3),
                                        (100, 9, 1)])
def test_step_tournament(m, n, elite):
    cfg = gao.Config(m=m, n=n, seed=3, elite=elite, mut_threshold=gao.rate_threshold(1, 2),
                     nc=2, nr=3)
    pop = gao.init_population(cfg)
    keys = gao.fitness(cfg, pop)
    for g in range(3):
        pop2, keys2 = gao.step(cfg, pop, keys, g)
        assert gao.check_invariants(pop2) == 0
        if elite:
            sel = gao.select_set(keys, elite)
            assert np.array_equal(pop2[:elite], pop[sel])
            assert np.array_equal(keys2[:elite], keys[sel])
        _children_consistent(cfg, pop, keys, pop2, keys2, g)
        assert np.array_equal(gao.fitness(cfg, pop2), keys2)
        pop, keys = pop2, keys2


def test_step_paper_mode():
    m, N = 12, 25
    cfg = gao.Config(m=m, n=4 * N, seed=8, selection=gao.SEL_PAPER, fitness=gao.FIT_F2,
                     xo_threshold=1 << 32, mut_threshold=1 << 32, nc=2, nr=2)
    pop = gao.init_population(cfg)
    keys = gao.fitness(cfg, pop)
    pop2, keys2 = gao.step(cfg, pop, keys, 0)
    sel = gao.select_set(keys, 2 * N)
    # the parents are exactly the best half, each once, in a shuffled order
    src = [gao.permute(cfg.seed, 1, 2 * N, s) for s in range(2 * N)]
    assert sorted(src) == list(range(2 * N))
    assert np.array_equal(pop2[: 2 * N], pop[sel[src]])
    assert np.array_equal(keys2[: 2 * N], keys[sel[src]])
    # offspring O_k and O_{N+k} come from (P_k, P_{k+N}) with a cut in [1, m-1]
    for k in range(N):
        A, B = pop2[k], pop2[k + N]
        for s in (2 * N + k, 3 * N + k):
            mixed = sum(not (np.array_equal(pop2[s][:, j], A[:, j]) or
                             np.array_equal(pop2[s][:, j], B[:, j])) for j in range(m))
            assert mixed <= cfg.nc
    assert gao.check_invariants(pop2) == 0
    assert np.array_equal(gao.fitness(cfg, pop2), keys2)
    assert keys2[: 2 * N].max() <= np.sort(keys)[2 * N - 1]


# --------------------------------------------------------------------------
# The pair operator of a generation: crossover cut, parent orientation, coins
# --------------------------------------------------------------------------
def _cut_of(A, B, C0, C1):
    """The cut c in [1, m-1] with C0 = A[:, <c] | B[:, >=c] and
    C1 = B[:, <c] | A[:, >=c], or None when no cut explains the children.
    Meant for parents whose columns 1..m-1 all differ, where such a cut is
    unique (column 0 is all +1 in both, so c = 0 would equal c = 1)."""
    m = A.shape[0]
    for c in range(1, m):
        if (np.array_equal(C0[:, :c], A[:, :c]) and np.array_equal(C0[:, c:], B[:, c:])
                and np.array_equal(C1[:, :c], B[:, :c]) and np.array_equal(C1[:, c:], A[:, c:])):
            return c
    return None


def _distinct_columns(A, B):
    return all(not np.array_equal(A[:, j], B[:, j]) for j in range(1, A.shape[0]))


def _tournament_pairs(cfg, pop, keys, gen_in):
    """(pair, parent a, parent b) of every child pair of a tournament step."""
    return [(p, *gao.tournament_parents(cfg, keys, gen_in + 1, p))
            for p in range((cfg.n - cfg.elite + 1) // 2)]


def _uniform_cut_ok(cuts, m):
    """Chi-square goodness of fit of the cuts to the uniform law on [1, m-1]."""
    counts = np.bincount(np.asarray(cuts), minlength=m)[1:]
    assert counts.sum() == len(cuts)
    return stats.chisquare(counts).pvalue > 1e-4


@pytest.mark.parametrize("m", [8, 20, 36])
def test_tournament_crossover_cut_range_and_orientation(m):
    """With the crossover coin always on and no mutation, child 0 of pair p
    is a[:, <c] | b[:, >=c] and child 1 the complement, for one cut c, where a
    is the parent of the first tournament and b of the second (Sec. 3.4:
    each part of one parent is joined with the adjoining part of the other);
    the cut is uniform over [1, m-1] (the listing's random_integers(1, m-1)).
    A swapped parent order, a missing complement, a cut range of [0, m-1]
    (c = 0 looks like c = 1 here and doubles its count) or [1, m-2] fails."""
    cfg = gao.Config(m=m, n=12000, seed=40 + m, xo_threshold=1 << 32, mut_threshold=0, nc=0,
                     nr=0, tournament_k=2)
    pop = inputs.random_population(m, cfg.n, seed=m)
    keys = gao.fitness(cfg, pop)
    pop2, _ = gao.step(cfg, pop, keys, 0)
    cuts = []
    for p, a, b in _tournament_pairs(cfg, pop, keys, 0):
        if a == b or not _distinct_columns(pop[a], pop[b]):
            continue
        c = _cut_of(pop[a], pop[b], pop2[2 * p], pop2[2 * p + 1])
        assert c is not None, p
        cuts.append(c)
    assert len(cuts) > 5000
    assert _uniform_cut_ok(cuts, m)


@pytest.mark.parametrize("m", [8, 20])
def test_paper_mode_crossover_orientation(m):
    """Paper mode (Sec. 3.4, the crossover figure): offspring slot 2N + k
    takes the columns before the cut from parent P_k and the rest from
    P_{k+N}; slot 3N + k takes the columns before the cut from P_{k+N}.  The
    cut is drawn for every pair, uniform over [1, m-1]."""
    N = 3000
    cfg = gao.Config(m=m, n=4 * N, seed=70 + m, selection=gao.SEL_PAPER, fitness=gao.FIT_F2,
                     xo_threshold=1 << 32, mut_threshold=0, nc=0, nr=0)
    pop = inputs.random_population(m, cfg.n, seed=100 + m)
    keys = gao.fitness(cfg, pop)
    pop2, _ = gao.step(cfg, pop, keys, 0)
    cuts = []
    for k in range(N):
        P, Q = pop2[k], pop2[k + N]
        if not _distinct_columns(P, Q):
            continue
        c = _cut_of(P, Q, pop2[2 * N + k], pop2[3 * N + k])
        assert c is not None, k
        cuts.append(c)
    assert len(cuts) > N // 2
    assert _uniform_cut_ok(cuts, m)


def test_no_crossover_no_mutation_children_copy_parents():
    """Both coins off: child 0 of pair p is parent a and child 1 parent b in
    tournament mode; in paper mode offspring 2N + k is P_k and 3N + k is
    P_{k+N}."""
    m = 12
    cfg = gao.Config(m=m, n=801, seed=5, xo_threshold=0, mut_threshold=0, nc=0, nr=0, elite=3)
    pop = inputs.random_population(m, cfg.n, seed=1)
    keys = gao.fitness(cfg, pop)
    pop2, keys2 = gao.step(cfg, pop, keys, 4)
    for p, a, b in _tournament_pairs(cfg, pop, keys, 4):
        for ch, par in ((0, a), (1, b)):
            s = cfg.elite + 2 * p + ch
            if s < cfg.n:
                assert np.array_equal(pop2[s], pop[par]) and keys2[s] == keys[par]
    N = 200
    pc = gao.Config(m=m, n=4 * N, seed=6, selection=gao.SEL_PAPER, xo_threshold=0,
                    mut_threshold=0, nc=0, nr=0)
    pop = inputs.random_population(m, pc.n, seed=2)
    keys = gao.fitness(pc, pop)
    pop2, _ = gao.step(pc, pop, keys, 0)
    assert np.array_equal(pop2[2 * N:3 * N], pop2[:N])
    assert np.array_equal(pop2[3 * N:], pop2[N:2 * N])


def _binomial_ok(count, trials, rate):
    return stats.binomtest(count, trials, rate).pvalue > 1e-4


@pytest.mark.parametrize("num,den", [(1, 2), (1, 10), (3, 4)])
def test_crossover_coin_rate(num, den):
    """The crossover coin of a pair succeeds with the configured rate (the
    benchmark configurations use 0.5): over pairs whose parents differ in
    every column, the fraction of pairs whose children are not the parents
    copied is binomial with that rate."""
    m = 16
    cfg = gao.Config(m=m, n=16000, seed=den, xo_threshold=gao.rate_threshold(num, den),
                     mut_threshold=0, nc=0, nr=0)
    pop = inputs.random_population(m, cfg.n, seed=7)
    keys = gao.fitness(cfg, pop)
    pop2, _ = gao.step(cfg, pop, keys, 2)
    crossed = trials = 0
    for p, a, b in _tournament_pairs(cfg, pop, keys, 2):
        if a == b or not _distinct_columns(pop[a], pop[b]):
            continue
        trials += 1
        same = np.array_equal(pop2[2 * p], pop[a]) and np.array_equal(pop2[2 * p + 1], pop[b])
        if not same:
            assert _cut_of(pop[a], pop[b], pop2[2 * p], pop2[2 * p + 1]) is not None
            crossed += 1
    assert trials > 7000
    assert _binomial_ok(crossed, trials, num / den), (crossed, trials)


@pytest.mark.parametrize("num,den", [(1, 10), (1, 2)])
def test_mutation_coin_rate_per_child(num, den):
    """Each child is mutated with the configured probability (0.1 in the
    benchmark configurations), independently of its sibling: with the
    crossover off and 64 row pairs per mutated child (a mutated column is
    then left unchanged with negligible probability), the children that
    differ from their parent are binomial with that rate, and both children
    of a pair are mutated at the rate's square."""
    m = 16
    cfg = gao.Config(m=m, n=20000, seed=11 + den, xo_threshold=0,
                     mut_threshold=gao.rate_threshold(num, den), nc=1, nr=64)
    pop = inputs.random_population(m, cfg.n, seed=8)
    keys = gao.fitness(cfg, pop)
    pop2, _ = gao.step(cfg, pop, keys, 0)
    changed, both, pairs = 0, 0, 0
    for p, a, b in _tournament_pairs(cfg, pop, keys, 0):
        c0 = not np.array_equal(pop2[2 * p], pop[a])
        c1 = not np.array_equal(pop2[2 * p + 1], pop[b])
        changed += c0 + c1
        both += c0 and c1
        pairs += 1
        for ch, par in ((0, a), (1, b)):
            diff = np.argwhere(pop2[2 * p + ch] != pop[par])
            assert len(set(diff[:, 1].tolist())) <= 1   # one column (nc = 1)
    rate = num / den
    assert _binomial_ok(changed, 2 * pairs, rate), (changed, 2 * pairs)
    assert _binomial_ok(both, pairs, rate * rate), (both, pairs)


def test_run_finds_hadamard_m4_and_m8():
    for m in (4, 8):
        cfg = gao.Config(m=m, n=256, seed=0, max_generations=200)
        res, pop, keys = gao.run(cfg)
        assert res["found"] and res["best_key"] == 0
        H = pop[res["index"]]
        assert hf.is_hadamard(H) and gao.check_invariants(H[None]) == 0
        assert keys[res["index"]] == 0 and keys.min() == 0
        assert res["index"] == int(np.nonzero(keys == 0)[0][0])


def test_run_deterministic_and_budgeted():
    cfg = gao.Config(m=20, n=64, seed=1, max_generations=7, stop_on_found=False)
    r1, p1, k1 = gao.run(cfg)
    r2, p2, k2 = gao.run(cfg)
    assert r1 == r2 and np.array_equal(p1, p2) and np.array_equal(k1, k2)
    assert r1["generation"] == 7


def test_run_equals_repeated_steps():
    cfg = gao.Config(m=12, n=40, seed=6, max_generations=5, stop_on_found=False, elite=2)
    pop = gao.init_population(cfg)
    keys = gao.fitness(cfg, pop)
    for g in range(5):
        pop, keys = gao.step(cfg, pop, keys, g)
    _, p, k = gao.run(cfg)
    assert np.array_equal(p, pop) and np.array_equal(k, keys)


@pytest.mark.parametrize("m,N,seed", [(12, 30, 5), (20, 16, 6), (68, 8, 7)])
def test_step_shared_mutation_one_pattern_per_generation(m, N, seed):
    """First mutation method (Sec. 3.5): every offspring of a generation is
    mutated at the same column and row pair, and flipped only where the two
    entries differ.  Compared with the same step without mutation (selection
    and crossover draw from other streams, so they are unchanged), each child
    differs in no entry or in the two entries of one +1/-1 pair, the pair is
    the same for the whole generation, and the unchanged children hold equal
    entries there.  Without the flag the children's pairs differ."""
    base = dict(m=m, n=4 * N, seed=seed, selection=gao.SEL_PAPER, fitness=gao.FIT_F2,
                xo_threshold=1 << 32, nc=1, nr=1)
    shared = gao.Config(**base, mut_threshold=1 << 32, mut_shared=True)
    own = gao.Config(**base, mut_threshold=1 << 32)
    plain = gao.Config(**base, mut_threshold=0)
    pop = gao.init_population(shared)
    keys = gao.fitness(shared, pop)

    def patterns(a, b):
        pats, same = set(), []
        for k in range(2 * N, 4 * N):
            pos = [tuple(x) for x in np.argwhere(a[k] != b[k])]
            if not pos:
                same.append(k)
                continue
            assert len(pos) == 2 and pos[0][1] == pos[1][1], pos  # one column
            (r1, c), (r2, _) = pos
            assert b[k][r1, c] == -b[k][r2, c]                   # a +1/-1 pair
            pats.add((r1, r2, c))
        return pats, same

    for g in range(3):
        a, ka = gao.step(shared, pop, keys, g)
        b, _ = gao.step(plain, pop, keys, g)
        assert np.array_equal(a[:2 * N], b[:2 * N])   # parents untouched
        pats, same = patterns(a, b)
        assert len(pats) == 1, pats
        (r1, r2, c), = pats
        for k in same:
            assert b[k][r1, c] == b[k][r2, c]
        assert np.array_equal(gao.fitness(shared, a), ka)
        o, _ = gao.step(own, pop, keys, g)
        assert len(patterns(o, b)[0]) > 1
        pop, keys = a, ka


def test_validate():
    ok = gao.Config(m=8, n=10)
    assert gao.validate(ok)
    bad = [
        dict(m=6), dict(m=0), dict(m=132), dict(n=1), dict(fitness=6),
        dict(selection=2), dict(tournament_k=0), dict(elite=10),
        dict(xo_threshold=(1 << 32) + 1), dict(nc=0), dict(nr=0),
        dict(selection=gao.SEL_PAPER, n=10), dict(selection=gao.SEL_PAPER, n=12, elite=1),
    ]
    for kw in bad:
        c = gao.Config(**{**ok.__dict__, **kw})
        assert not gao.validate(c), kw
    assert gao.validate(gao.Config(m=8, n=10, mut_threshold=0, nc=0, nr=0))
    assert gao.validate(gao.Config(m=128, n=10)) and gao.validate(gao.Config(m=68, n=10))


@pytest.mark.slow
def test_paper_mode_search_band_m12():
    """Paper mode at m=12 (Table 3: 32-66 mean generations for NC, NR in
    1..4; population size unstated, the listing's default is N=1000).  A run
    either solves within a few hundred generations or stalls at a small
    positive F2 with a homogeneous parent half, as Sec. 4.1 describes."""
    solved = 0
    for seed in range(3):
        cfg = gao.Config(m=12, n=4000, seed=seed, selection=gao.SEL_PAPER, fitness=gao.FIT_F2,
                         xo_threshold=1 << 32, mut_threshold=1 << 32, nc=1, nr=2,
                         max_generations=400)
        res, pop, keys = gao.run(cfg)
        if res["found"]:
            solved += 1
            assert hf.is_hadamard(pop[res["index"]])
            assert res["generation"] <= 400
        else:
            assert res["best_key"] <= 8
    assert solved >= 2
