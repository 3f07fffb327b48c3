"""Helpers of the GPU tests: device tensors, layout conversion, config
mirroring between the library's config and the oracle's."""
import numpy as np
import pytest

import paper_2208_14961_amd as ga
from oracle import gao
from tests import inputs


def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def to_oracle(cfg: ga.Config) -> gao.Config:
    return gao.Config(m=cfg.m, n=cfg.n, seed=cfg.seed, fitness=cfg.fitness,
                      selection=cfg.selection, tournament_k=cfg.tournament_k,
                      elite=cfg.elite, xo_threshold=cfg.xo_threshold,
                      mut_threshold=cfg.mut_threshold, nc=cfg.nc, nr=cfg.nr,
                      max_generations=cfg.max_generations,
                      stop_on_found=bool(cfg.flags & ga.STOP_ON_FOUND),
                      mut_shared=bool(cfg.flags & ga.MUT_SHARED))


def dev_pop_from_int8(pop: np.ndarray):
    torch = torch_cuda()
    packed = inputs.pack(pop).view(np.int32)
    return torch.from_numpy(np.ascontiguousarray(packed)).cuda()


def int8_from_dev_pop(t, m: int) -> np.ndarray:
    torch_cuda().cuda.synchronize()
    return inputs.unpack(t.cpu().numpy().view(np.uint32), m)


def empty_pop(cfg: ga.Config):
    torch = torch_cuda()
    return torch.zeros(ga.pop_shape(cfg), dtype=torch.int32, device="cuda")


def empty_keys(cfg: ga.Config):
    torch = torch_cuda()
    return torch.zeros((cfg.n,), dtype=torch.int32, device="cuda")


def keys_np(t) -> np.ndarray:
    torch_cuda().cuda.synchronize()
    return t.cpu().numpy().view(np.uint32)


def announce(*what):
    print("CASE", *what, flush=True)
