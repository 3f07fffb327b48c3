"""Python binding of libga: the MI355X (gfx950) hot path of the genetic
algorithm for Hadamard matrices (Balogh & Ruiz, arXiv 2208.14961).

Each function marshals its arguments and calls the C ABI of the same name
(include/ga.h); every step of the computation runs in libga's HIP kernels.
Device buffers are torch tensors on a ROCm device:

* a population is an int32 tensor of shape (n, m, W), W = col_words(m)
  (1 up to order 32, 2 up to 64, 4 up to 128), holding the packed uint32
  words (bit r of column j set iff entry (r, j) is -1);
* keys are int32 tensors of shape (n,) (all keys are below 2^31);
* components are int32 tensors of shape (n, 3): (SQ, ABS, NNZ).

Calls are enqueued on torch's current stream unless a stream is given.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field, asdict
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libga.so")

GA_OK, GA_PENDING = 0, 1
GA_EINVAL, GA_ENOMEM, GA_EDEVICE, GA_EBUDGET, GA_ENOTFOUND, GA_ESTOPPED = -1, -2, -3, -4, -5, -6
FIT_SQ, FIT_ABS, FIT_NNZ, FIT_SQ_PLUS_NNZ, FIT_F1, FIT_F2 = range(6)
SEL_TOURNAMENT, SEL_PAPER = 0, 1
STOP_ON_FOUND = 1
MUT_SHARED = 2  # first mutation method of Sec. 3.5: one draw set per generation
MAX_ORDER = 128  # largest order m the library accepts (GA_MAX_M)
LANES_SHIFT = 8
# Gram products of ga_fitness / ga_fitness_repeat: xor + popcount, or the
# int8 matrix cores (orders 36..128); neither flag: the library's table.
GRAM_PACKED = 1 << 13
GRAM_MFMA = 2 << 13
MFMA_MIN_ORDER = 36


def col_words(m: int) -> int:
    """Words per packed column of order m (the layout of include/ga.h)."""
    return 1 if m <= 32 else (2 if m <= 64 else 4)


def lanes_flag(lanes: int) -> int:
    """flags bits forcing the children kernel's lanes per child (0: tuned)."""
    return lanes << LANES_SHIFT


class GAError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"libga status {status}: {message}")
        self.status = status


class _Config(ctypes.Structure):
    _fields_ = [
        ("m", ctypes.c_uint32), ("n", ctypes.c_uint32), ("seed", ctypes.c_uint64),
        ("fitness", ctypes.c_uint32), ("selection", ctypes.c_uint32),
        ("tournament_k", ctypes.c_uint32), ("elite", ctypes.c_uint32),
        ("xo_threshold", ctypes.c_uint64), ("mut_threshold", ctypes.c_uint64),
        ("nc", ctypes.c_uint32), ("nr", ctypes.c_uint32),
        ("max_generations", ctypes.c_uint32), ("flags", ctypes.c_uint32),
    ]


class _Result(ctypes.Structure):
    _fields_ = [
        ("found", ctypes.c_int32), ("generation", ctypes.c_uint32),
        ("index", ctypes.c_uint32), ("best_key", ctypes.c_uint32),
        ("matrix", ctypes.c_int8 * (MAX_ORDER * MAX_ORDER)),
    ]


def rate_threshold(num: int, den: int) -> int:
    """Coin threshold of a rate num/den: floor(num * 2^32 / den)."""
    return (num << 32) // den


@dataclass
class Config:
    """Mirror of ga_config; defaults are the plain GA of the benchmark
    configurations (binary tournament, crossover 0.5, one pair-flip per
    child at rate 0.1)."""
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
    flags: int = STOP_ON_FOUND

    @property
    def words(self) -> int:
        """Words per packed column: 1 up to order 32, 2 up to 64, 4 above."""
        return col_words(self.m)

    def c(self) -> _Config:
        return _Config(self.m, self.n, self.seed, self.fitness, self.selection,
                       self.tournament_k, self.elite, self.xo_threshold,
                       self.mut_threshold, self.nc, self.nr, self.max_generations,
                       self.flags)


_lib = None


def lib() -> ctypes.CDLL:
    """Loads libga.so; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2208_14961_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        P, vp = ctypes.POINTER, ctypes.c_void_p
        u32, u64, i32 = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
        sig = {
            "ga_last_error": (ctypes.c_char_p, []),
            "ga_validate": (i32, [P(_Config)]),
            "ga_population_words": (ctypes.c_size_t, [P(_Config)]),
            "ga_init_population": (i32, [P(_Config), vp, vp]),
            "ga_fitness": (i32, [P(_Config), vp, vp, vp, vp]),
            "ga_fitness_repeat": (i32, [P(_Config), vp, vp, u32, vp]),
            "ga_tuned_lanes": (u32, [P(_Config)]),
            "ga_step": (i32, [P(_Config), vp, vp, vp, vp, u32, vp]),
            "ga_step_static": (i32, [P(_Config), vp, vp, vp, vp, u32, vp]),
            "ga_paper_select": (i32, [P(_Config), vp, vp, vp, vp]),
            "ga_run": (i32, [P(_Config), vp, vp, vp, vp, P(_Result), vp]),
            "ga_run_batch": (i32, [P(_Config), u32, P(_Result), vp]),
            "ga_check_invariants": (i32, [P(_Config), vp, P(u32), vp]),
            "ga_pack": (i32, [P(_Config), vp, vp, vp, vp]),
            "ga_unpack": (i32, [P(_Config), vp, vp, vp]),
            "ga_server_create": (i32, [u64, i32, P(vp)]),
            "ga_submit": (i32, [vp, P(_Config), P(u64)]),
            "ga_poll": (i32, [vp, u64, P(_Result)]),
            "ga_wait": (i32, [vp, u64, P(_Result)]),
            "ga_request_latency": (i32, [vp, u64, P(ctypes.c_double)]),
            "ga_server_stop": (i32, [vp]),
            "ga_server_destroy": (i32, [vp]),
            "ga_timing_enable": (i32, [i32]),
            "ga_timing_read": (i32, [P(ctypes.c_double), P(u64)]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(status: int) -> int:
    if status < 0:
        raise GAError(status, lib().ga_last_error().decode())
    return status


def _stream(stream) -> ctypes.c_void_p:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dev(t, shape, name) -> ctypes.c_void_p:
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != torch.int32 or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous int32 tensor")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return ctypes.c_void_p(t.data_ptr())


def _result(r: _Result, m: int) -> dict:
    mat = np.frombuffer(bytes(r.matrix), dtype=np.int8)[: m * m].reshape(m, m).copy()
    return dict(found=bool(r.found), generation=int(r.generation), index=int(r.index),
                best_key=int(r.best_key), matrix=mat)


def pop_shape(cfg: Config):
    return (cfg.n, cfg.m, cfg.words)


def ga_validate(cfg: Config) -> bool:
    return lib().ga_validate(ctypes.byref(cfg.c())) == GA_OK


def ga_population_words(cfg: Config) -> int:
    return int(lib().ga_population_words(ctypes.byref(cfg.c())))


def ga_init_population(cfg: Config, pop, stream=None) -> None:
    _check(lib().ga_init_population(ctypes.byref(cfg.c()), _dev(pop, pop_shape(cfg), "pop"),
                                    _stream(stream)))


def ga_fitness(cfg: Config, pop, keys, comps=None, stream=None) -> None:
    cp = _dev(comps, (cfg.n, 3), "comps") if comps is not None else None
    _check(lib().ga_fitness(ctypes.byref(cfg.c()), _dev(pop, pop_shape(cfg), "pop"),
                            _dev(keys, (cfg.n,), "keys"), cp, _stream(stream)))


def ga_tuned_lanes(cfg: Config) -> int:
    """Lanes per child ga_run would use now for cfg (0 if cfg is invalid)."""
    return int(lib().ga_tuned_lanes(ctypes.byref(cfg.c())))


def ga_fitness_repeat(cfg: Config, pop, keys, reps: int, stream=None) -> None:
    _check(lib().ga_fitness_repeat(ctypes.byref(cfg.c()), _dev(pop, pop_shape(cfg), "pop"),
                                   _dev(keys, (cfg.n,), "keys"), reps, _stream(stream)))


def ga_step(cfg: Config, pop_in, keys_in, pop_out, keys_out, gen_in: int,
            stream=None) -> None:
    sh = pop_shape(cfg)
    _check(lib().ga_step(ctypes.byref(cfg.c()), _dev(pop_in, sh, "pop_in"),
                         _dev(keys_in, (cfg.n,), "keys_in"), _dev(pop_out, sh, "pop_out"),
                         _dev(keys_out, (cfg.n,), "keys_out"), gen_in, _stream(stream)))


def ga_step_static(cfg: Config, pop_in, keys_in, pop_out, keys_out, gen_in: int,
                   stream=None) -> None:
    """ga_step on the library's fixed device workspace: no allocation."""
    sh = pop_shape(cfg)
    _check(lib().ga_step_static(ctypes.byref(cfg.c()), _dev(pop_in, sh, "pop_in"),
                                _dev(keys_in, (cfg.n,), "keys_in"), _dev(pop_out, sh, "pop_out"),
                                _dev(keys_out, (cfg.n,), "keys_out"), gen_in, _stream(stream)))


def ga_paper_select(cfg: Config, keys, threshold, sel, stream=None) -> None:
    """Paper-mode truncation selection of one generation's keys (n <= 65536):
    sel (int32, n/2) gets the selected indices in increasing order; threshold
    (int32, 1) holds the previous threshold or -1 and gets this one."""
    _check(lib().ga_paper_select(ctypes.byref(cfg.c()), _dev(keys, (cfg.n,), "keys"),
                                 _dev(threshold, (1,), "threshold"),
                                 _dev(sel, (cfg.n // 2,), "sel"), _stream(stream)))


def ga_run(cfg: Config, pop_a, pop_b, keys_a, keys_b, stream=None) -> dict:
    sh = pop_shape(cfg)
    r = _Result()
    _check(lib().ga_run(ctypes.byref(cfg.c()), _dev(pop_a, sh, "pop_a"),
                        _dev(pop_b, sh, "pop_b"), _dev(keys_a, (cfg.n,), "keys_a"),
                        _dev(keys_b, (cfg.n,), "keys_b"), ctypes.byref(r), _stream(stream)))
    return _result(r, cfg.m)


def ga_run_batch(cfgs: Sequence[Config], stream=None) -> list:
    arr = (_Config * len(cfgs))(*[c.c() for c in cfgs])
    res = (_Result * len(cfgs))()
    _check(lib().ga_run_batch(arr, len(cfgs), res, _stream(stream)))
    return [_result(res[i], cfgs[i].m) for i in range(len(cfgs))]


def _dev8(t, shape, name) -> ctypes.c_void_p:
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != torch.int8 or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous int8 tensor")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return ctypes.c_void_p(t.data_ptr())


def ga_pack(cfg: Config, q, pop, bad=None, stream=None) -> None:
    """int8 matrices q (n, m, m), +1/-1, into the packed population pop;
    bad: None or an int32 device tensor of shape (1,) increased by the
    number of entries other than +1 and -1."""
    b = ctypes.c_void_p(None) if bad is None else _dev(bad, (1,), "bad")
    _check(lib().ga_pack(ctypes.byref(cfg.c()), _dev8(q, (cfg.n, cfg.m, cfg.m), "q"),
                         _dev(pop, pop_shape(cfg), "pop"), b, _stream(stream)))


def ga_unpack(cfg: Config, pop, q, stream=None) -> None:
    """The packed population pop as int8 matrices q (n, m, m) of +1/-1."""
    _check(lib().ga_unpack(ctypes.byref(cfg.c()), _dev(pop, pop_shape(cfg), "pop"),
                           _dev8(q, (cfg.n, cfg.m, cfg.m), "q"), _stream(stream)))


def ga_check_invariants(cfg: Config, pop, stream=None) -> int:
    bad = ctypes.c_uint32()
    _check(lib().ga_check_invariants(ctypes.byref(cfg.c()), _dev(pop, pop_shape(cfg), "pop"),
                                     ctypes.byref(bad), _stream(stream)))
    return int(bad.value)


def ga_timing_enable(on: bool) -> None:
    _check(lib().ga_timing_enable(1 if on else 0))


def ga_timing_read():
    """(mean time per generation in ms, generations) of the ga_run
    generation loops timed since ga_timing_enable(True)."""
    ms = ctypes.c_double()
    n = ctypes.c_uint64()
    _check(lib().ga_timing_read(ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


class Server:
    """ga_server_create / ga_submit / ga_poll / ga_wait / ga_server_stop /
    ga_server_destroy."""

    def __init__(self, hbm_budget_bytes: int, device: int = 0):
        self._h = ctypes.c_void_p()
        _check(lib().ga_server_create(hbm_budget_bytes, device, ctypes.byref(self._h)))
        self._m = {}

    def submit(self, cfg: Config) -> int:
        rid = ctypes.c_uint64()
        _check(lib().ga_submit(self._h, ctypes.byref(cfg.c()), ctypes.byref(rid)))
        self._m[rid.value] = cfg.m
        return rid.value

    def poll(self, rid: int) -> Optional[dict]:
        r = _Result()
        st = _check(lib().ga_poll(self._h, rid, ctypes.byref(r)))
        return None if st == GA_PENDING else _result(r, self._m[rid])

    def wait(self, rid: int) -> dict:
        r = _Result()
        _check(lib().ga_wait(self._h, rid, ctypes.byref(r)))
        return _result(r, self._m[rid])

    def latency(self, rid: int) -> float:
        s = ctypes.c_double()
        _check(lib().ga_request_latency(self._h, rid, ctypes.byref(s)))
        return s.value

    def stop(self) -> None:
        """Stops the worker: unfinished requests fail with GA_ESTOPPED, and
        later submissions are refused; finished results stay readable."""
        _check(lib().ga_server_stop(self._h))

    def close(self) -> None:
        if self._h:
            _check(lib().ga_server_destroy(self._h))
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
