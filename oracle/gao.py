"""ctypes wrapper of the CPU oracle (``oracle/gao.c``).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark use it to check and time the GPU library.  The product path
never imports this module.

Populations are numpy int8 arrays of shape ``(n, m, m)`` with entries +1/-1,
entry ``[k, i, j]`` being row i, column j of matrix k (paper, Sec. 3.4).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gao.c")
_LIB = os.path.join(_HERE, "libgao.so")

FIT_SQ, FIT_ABS, FIT_NNZ, FIT_SQ_PLUS_NNZ, FIT_F1, FIT_F2 = range(6)
SEL_TOURNAMENT, SEL_PAPER = 0, 1
STREAM_INIT, STREAM_SELECT, STREAM_XOVER, STREAM_MUTATE, STREAM_PERM = 1, 2, 3, 4, 5


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (OpenMP over individuals)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < max(
        os.path.getmtime(_SRC), os.path.getmtime(os.path.join(_HERE, "gao.h"))
    ):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall",
             "-Wextra", _SRC, "-o", tmp]
        )
        os.replace(tmp, _LIB)
    return _LIB


class _Config(ctypes.Structure):
    _fields_ = [
        ("m", ctypes.c_uint32),
        ("n", ctypes.c_uint32),
        ("seed", ctypes.c_uint64),
        ("fitness", ctypes.c_uint32),
        ("selection", ctypes.c_uint32),
        ("tournament_k", ctypes.c_uint32),
        ("elite", ctypes.c_uint32),
        ("xo_threshold", ctypes.c_uint64),
        ("mut_threshold", ctypes.c_uint64),
        ("nc", ctypes.c_uint32),
        ("nr", ctypes.c_uint32),
        ("max_generations", ctypes.c_uint32),
        ("stop_on_found", ctypes.c_uint32),
        ("mut_shared", ctypes.c_uint32),
    ]


class _Result(ctypes.Structure):
    _fields_ = [
        ("found", ctypes.c_int32),
        ("generation", ctypes.c_uint32),
        ("index", ctypes.c_uint32),
        ("best_key", ctypes.c_uint32),
    ]


def rate_threshold(num: int, den: int) -> int:
    """Bernoulli threshold for a rate num/den: floor(num * 2^32 / den)."""
    return (num << 32) // den


@dataclass
class Config:
    m: int
    n: int
    seed: int = 0
    fitness: int = FIT_SQ
    selection: int = SEL_TOURNAMENT
    tournament_k: int = 2
    elite: int = 0
    xo_threshold: int = 1 << 31
    mut_threshold: int = rate_threshold(1, 10)
    nc: int = 1
    nr: int = 1
    max_generations: int = 100
    stop_on_found: bool = True
    mut_shared: bool = False  # first mutation method of Sec. 3.5

    def c(self) -> _Config:
        return _Config(self.m, self.n, self.seed, self.fitness, self.selection,
                       self.tournament_k, self.elite, self.xo_threshold,
                       self.mut_threshold, self.nc, self.nr,
                       self.max_generations, int(bool(self.stop_on_found)),
                       int(bool(self.mut_shared)))


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        P = ctypes.POINTER
        u32, u64, i32 = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
        vp = ctypes.c_void_p
        sig = {
            "gao_validate": (i32, [P(_Config)]),
            "gao_philox4x32_10": (None, [vp, vp, vp]),
            "gao_draw": (u32, [u64, u32, u32, u32, u32]),
            "gao_bounded": (u32, [u32, u32]),
            "gao_gram": (None, [u32, vp, vp]),
            "gao_fitness_one": (u32, [u32, u32, vp, vp]),
            "gao_fitness": (i32, [P(_Config), vp, vp, vp]),
            "gao_init_population": (i32, [P(_Config), vp]),
            "gao_crossover": (None, [u32, vp, vp, u32, vp, vp]),
            "gao_mutate": (None, [u32, vp, u32, vp, u32, vp, vp]),
            "gao_permute": (u32, [u64, u32, u32, u32]),
            "gao_select_set": (None, [vp, u32, u32, vp]),
            "gao_tournament_parents": (None, [P(_Config), vp, u32, u32, vp, vp]),
            "gao_step": (i32, [P(_Config), vp, vp, vp, vp, u32]),
            "gao_run": (i32, [P(_Config), vp, vp, P(_Result)]),
            "gao_check_invariants": (u32, [u32, u32, vp]),
            "gao_num_threads": (i32, []),
            "gao_set_num_threads": (None, [i32]),
        }
        for name, (res, args) in sig.items():
            f = getattr(_lib, name)
            f.restype = res
            f.argtypes = args
    return _lib


def _ptr(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.c_void_p)


def validate(cfg: Config) -> bool:
    return lib().gao_validate(ctypes.byref(cfg.c())) == 0


def philox(ctr, key) -> np.ndarray:
    c = np.asarray(ctr, dtype=np.uint32).copy()
    k = np.asarray(key, dtype=np.uint32).copy()
    out = np.zeros(4, dtype=np.uint32)
    lib().gao_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def draw(seed: int, stream: int, gen: int, idx: int, d: int) -> int:
    return lib().gao_draw(seed, stream, gen, idx, d)


def bounded(u: int, r: int) -> int:
    return lib().gao_bounded(u, r)


def gram(Q: np.ndarray) -> np.ndarray:
    Q = np.ascontiguousarray(Q, dtype=np.int8)
    m = Q.shape[0]
    G = np.zeros((m, m), dtype=np.int32)
    lib().gao_gram(m, _ptr(Q), _ptr(G))
    return G


def fitness_one(Q: np.ndarray, kind: int = FIT_SQ):
    """Returns (key, (SQ, ABS, NNZ)) of one matrix."""
    Q = np.ascontiguousarray(Q, dtype=np.int8)
    comps = np.zeros(3, dtype=np.uint32)
    key = lib().gao_fitness_one(Q.shape[0], kind, _ptr(Q), _ptr(comps))
    return int(key), tuple(int(x) for x in comps)


def fitness(cfg: Config, pop: np.ndarray, with_comps: bool = False):
    pop = np.ascontiguousarray(pop, dtype=np.int8)
    keys = np.zeros(cfg.n, dtype=np.uint32)
    comps = np.zeros((cfg.n, 3), dtype=np.uint32) if with_comps else None
    rc = lib().gao_fitness(ctypes.byref(cfg.c()), _ptr(pop), _ptr(keys),
                           _ptr(comps) if with_comps else None)
    if rc:
        raise ValueError("invalid oracle configuration")
    return (keys, comps) if with_comps else keys


def init_population(cfg: Config) -> np.ndarray:
    pop = np.zeros((cfg.n, cfg.m, cfg.m), dtype=np.int8)
    if lib().gao_init_population(ctypes.byref(cfg.c()), _ptr(pop)):
        raise ValueError("invalid oracle configuration")
    return pop


def crossover(A: np.ndarray, B: np.ndarray, cut: int):
    A = np.ascontiguousarray(A, dtype=np.int8)
    B = np.ascontiguousarray(B, dtype=np.int8)
    O0 = np.zeros_like(A)
    O1 = np.zeros_like(A)
    lib().gao_crossover(A.shape[0], _ptr(A), _ptr(B), cut, _ptr(O0), _ptr(O1))
    return O0, O1


def mutate(Q: np.ndarray, cols, r1, r2) -> np.ndarray:
    Q = np.ascontiguousarray(Q, dtype=np.int8).copy()
    c = np.asarray(cols, dtype=np.uint32)
    a = np.asarray(r1, dtype=np.uint32)
    b = np.asarray(r2, dtype=np.uint32)
    assert a.shape == b.shape
    lib().gao_mutate(Q.shape[0], _ptr(Q), len(c), _ptr(c), len(a), _ptr(a), _ptr(b))
    return Q


def permute(seed: int, gen: int, domain: int, s: int) -> int:
    return lib().gao_permute(seed, gen, domain, s)


def select_set(keys: np.ndarray, count: int) -> np.ndarray:
    keys = np.ascontiguousarray(keys, dtype=np.uint32)
    out = np.zeros(count, dtype=np.uint32)
    lib().gao_select_set(_ptr(keys), len(keys), count, _ptr(out))
    return out


def tournament_parents(cfg: Config, keys: np.ndarray, gen_out: int, p: int):
    keys = np.ascontiguousarray(keys, dtype=np.uint32)
    a = ctypes.c_uint32()
    b = ctypes.c_uint32()
    lib().gao_tournament_parents(ctypes.byref(cfg.c()), _ptr(keys), gen_out, p,
                                 ctypes.byref(a), ctypes.byref(b))
    return a.value, b.value


def step(cfg: Config, pop: np.ndarray, keys: np.ndarray, gen_in: int):
    pop = np.ascontiguousarray(pop, dtype=np.int8)
    keys = np.ascontiguousarray(keys, dtype=np.uint32)
    pop_out = np.zeros_like(pop)
    keys_out = np.zeros_like(keys)
    if lib().gao_step(ctypes.byref(cfg.c()), _ptr(pop), _ptr(keys),
                      _ptr(pop_out), _ptr(keys_out), gen_in):
        raise ValueError("invalid oracle configuration")
    return pop_out, keys_out


def run(cfg: Config):
    """Whole run from generation 0; returns (result dict, final pop, keys)."""
    pop = np.zeros((cfg.n, cfg.m, cfg.m), dtype=np.int8)
    keys = np.zeros(cfg.n, dtype=np.uint32)
    res = _Result()
    if lib().gao_run(ctypes.byref(cfg.c()), _ptr(pop), _ptr(keys),
                     ctypes.byref(res)):
        raise ValueError("invalid oracle configuration")
    out = dict(found=bool(res.found), generation=res.generation,
               index=res.index, best_key=res.best_key)
    return out, pop, keys


def check_invariants(pop: np.ndarray) -> int:
    pop = np.ascontiguousarray(pop, dtype=np.int8)
    return int(lib().gao_check_invariants(pop.shape[1], pop.shape[0], _ptr(pop)))


def num_threads() -> int:
    return int(lib().gao_num_threads())


def set_num_threads(threads: int) -> None:
    """Threads of the oracle's loops over individuals (results do not
    depend on it)."""
    lib().gao_set_num_threads(int(threads))
