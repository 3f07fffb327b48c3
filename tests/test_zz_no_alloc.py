"""ga_step_static (no device allocation, a fixed workspace array) against
ga_step: bit-identical generations on two calls in a row, the second with a
smaller population, for elitist and paper-mode selection (the paths that use
the workspace) and a plain tournament."""
import numpy as np
import pytest

import paper_2208_14961_amd as ga
from tests.gpu_util import announce, empty_keys, empty_pop, int8_from_dev_pop, keys_np, torch_cuda

pytestmark = pytest.mark.gpu


def _both(cfg: ga.Config, gen_in: int):
    """The same generation from ga_step and ga_step_static."""
    pop, keys = empty_pop(cfg), empty_keys(cfg)
    ga.ga_init_population(cfg, pop)
    ga.ga_fitness(cfg, pop, keys)
    outs = []
    for fn in (ga.ga_step, ga.ga_step_static):
        po, ko = empty_pop(cfg), empty_keys(cfg)
        fn(cfg, pop, keys, po, ko, gen_in)
        outs.append((int8_from_dev_pop(po, cfg.m), keys_np(ko)))
    (p0, k0), (p1, k1) = outs
    assert np.array_equal(k0, k1)
    assert np.array_equal(p0, p1)
    return k1


@pytest.mark.parametrize("first,second", [
    (ga.Config(m=20, n=40000, seed=3, elite=400, fitness=ga.FIT_SQ, flags=0),
     ga.Config(m=12, n=3000, seed=4, selection=ga.SEL_PAPER, fitness=ga.FIT_F2,
               xo_threshold=1 << 32, mut_threshold=1 << 32, nc=2, nr=2)),
    (ga.Config(m=36, n=20000, seed=5, selection=ga.SEL_PAPER, fitness=ga.FIT_F1,
               xo_threshold=1 << 32, mut_threshold=1 << 32, nc=3, nr=2),
     ga.Config(m=32, n=5000, seed=6, elite=50, fitness=ga.FIT_SQ_PLUS_NNZ)),
    (ga.Config(m=8, n=4096, seed=7),
     ga.Config(m=100, n=999, seed=8, elite=9, fitness=ga.FIT_F2)),
])
def test_step_static_equals_step(first, second):
    torch_cuda()
    for cfg, gen_in in ((first, 0), (second, 5)):
        announce("step static", cfg.m, cfg.n, cfg.selection, cfg.elite, gen_in)
        _both(cfg, gen_in)


def test_step_static_rejects_bad_arguments():
    torch_cuda()
    cfg = ga.Config(m=8, n=100)
    a, b = empty_pop(cfg), empty_keys(cfg)
    with pytest.raises(ga.GAError) as e:
        ga.ga_step_static(cfg, a, b, a, empty_keys(cfg), 0)
    assert e.value.status == ga.GA_EINVAL
