"""Seeded synthetic workloads (inputs only).

Builds ground-truth networks and simulates spike rasters from the
discrete-time exponential-link GLM (the paper's validation protocol, Fig. 2,
with the network structures of Sec. 3.1 and Sec. 3.4).  Nothing here
evaluates a likelihood or a gradient: the FP64 oracle and the GPU library
both take these rasters as input.

The native part lives in ``gen.c`` (Philox4x32-10 counter-based draws, so a
result depends only on the seed).  ``build()`` compiles it with gcc.
"""
from __future__ import annotations

import ctypes
import dataclasses
import math
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.c")
_LIB = os.path.join(_HERE, "_synth.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile gen.c into _synth.so (gcc, OpenMP, no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
               "-fno-fast-math", "-std=c11", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build(force=True)
    lib = ctypes.CDLL(_LIB)
    P = ctypes.POINTER
    c_dp = P(ctypes.c_double)
    lib.synth_philox4x32_10.argtypes = [P(ctypes.c_uint32)] * 3
    lib.synth_net_bernoulli.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                        ctypes.c_double, ctypes.c_double, ctypes.c_uint64, c_dp]
    lib.synth_net_fixed_indegree.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                             ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                             ctypes.c_uint64, c_dp]
    lib.synth_net_fixed_indegree.restype = ctypes.c_int
    lib.synth_net_synfire.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                      ctypes.c_double, ctypes.c_double, ctypes.c_int32,
                                      ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_uint64, c_dp, P(ctypes.c_int32)]
    lib.synth_net_synfire.restype = ctypes.c_int
    lib.synth_rates_uniform.argtypes = [ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                        ctypes.c_uint64, c_dp]
    lib.synth_uniform_ints.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                                       ctypes.c_uint64, ctypes.c_uint32, P(ctypes.c_int64)]
    lib.synth_simulate.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_double,
                                   ctypes.c_double, c_dp, c_dp, ctypes.c_uint64, ctypes.c_int]
    lib.synth_simulate.restype = ctypes.c_int64
    lib.synth_take.argtypes = [P(ctypes.c_int64), P(ctypes.c_int32)]
    _lib = lib
    return lib


def _ptr(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def philox4x32_10(ctr, key):
    """Raw Philox4x32-10 block (for the known-answer test)."""
    lib = _load()
    c = np.asarray(ctr, dtype=np.uint32).copy()
    k = np.asarray(key, dtype=np.uint32).copy()
    o = np.zeros(4, dtype=np.uint32)
    lib.synth_philox4x32_10(_ptr(c, ctypes.c_uint32), _ptr(k, ctypes.c_uint32),
                            _ptr(o, ctypes.c_uint32))
    return o


@dataclasses.dataclass
class Recording:
    """One synthetic recording: raster + ground truth."""
    name: str
    n_neurons: int
    n_bins: int
    dt: float            # bin width [s]
    tau: float           # true kernel time constant [s]
    bins: np.ndarray     # int64 [q], sorted by (bin, neuron)
    neurons: np.ndarray  # int32 [q]
    J: np.ndarray        # float64 [N, N], J[i, j] = weight j -> i
    mu: np.ndarray       # float64 [N], log base rate (1/s)
    n_exc: int
    seed: int
    group_of: Optional[np.ndarray] = None  # synfire group per neuron (-1 = none)

    @property
    def T(self) -> float:
        return self.n_bins * self.dt

    @property
    def n_spikes(self) -> int:
        return int(self.bins.shape[0])

    def counts(self) -> np.ndarray:
        return np.bincount(self.neurons, minlength=self.n_neurons).astype(np.int64)


def event_times(rec: Recording, seed: int = 0):
    """Continuous spike times of a raster: each spike of bin b is placed at
    (b + u) dt with u uniform in [0, 1), then the events are sorted by (time,
    neuron).  Returns (times [q] float64 seconds in [0, T), neurons [q] int32)."""
    rng = np.random.default_rng(seed)
    t = (rec.bins.astype(np.float64) + rng.random(rec.bins.shape[0])) * rec.dt
    order = np.lexsort((rec.neurons, t))
    return np.ascontiguousarray(t[order]), np.ascontiguousarray(rec.neurons[order])


def simulate(N: int, B: int, dt: float, tau: float, mu: np.ndarray, J: np.ndarray,
             seed: int, threads: int = 0):
    lib = _load()
    mu = np.ascontiguousarray(mu, dtype=np.float64)
    J = np.ascontiguousarray(J, dtype=np.float64)
    n = lib.synth_simulate(int(N), int(B), float(dt), float(tau), _ptr(mu, ctypes.c_double),
                           _ptr(J, ctypes.c_double), ctypes.c_uint64(seed), int(threads))
    if n < 0:
        raise RuntimeError(f"synth_simulate failed ({n})")
    bins = np.empty(n, dtype=np.int64)
    neu = np.empty(n, dtype=np.int32)
    lib.synth_take(_ptr(bins, ctypes.c_int64), _ptr(neu, ctypes.c_int32))
    return bins, neu


def net_bernoulli(N, n_exc, p, j_exc, j_inh, seed):
    lib = _load()
    J = np.zeros((N, N), dtype=np.float64)
    lib.synth_net_bernoulli(N, n_exc, p, j_exc, j_inh, ctypes.c_uint64(seed),
                            _ptr(J, ctypes.c_double))
    return J


def net_fixed_indegree(N, n_exc, k_exc, k_inh, j_exc, j_inh, seed):
    lib = _load()
    J = np.zeros((N, N), dtype=np.float64)
    rc = lib.synth_net_fixed_indegree(N, n_exc, k_exc, k_inh, j_exc, j_inh,
                                      ctypes.c_uint64(seed), _ptr(J, ctypes.c_double))
    if rc != 0:
        raise ValueError(f"fixed in-degree network impossible (rc={rc})")
    return J


def net_synfire(N, n_exc, p_bg, j_exc, j_inh, n_groups, group_size, p_chain, j_chain, seed):
    lib = _load()
    J = np.zeros((N, N), dtype=np.float64)
    g = np.zeros(N, dtype=np.int32)
    rc = lib.synth_net_synfire(N, n_exc, p_bg, j_exc, j_inh, n_groups, group_size, p_chain,
                               j_chain, ctypes.c_uint64(seed), _ptr(J, ctypes.c_double),
                               _ptr(g, ctypes.c_int32))
    if rc != 0:
        raise ValueError(f"synfire network impossible (rc={rc})")
    return J, g


def rates_uniform(N, lo, hi, seed):
    lib = _load()
    r = np.zeros(N, dtype=np.float64)
    lib.synth_rates_uniform(N, lo, hi, ctypes.c_uint64(seed), _ptr(r, ctypes.c_double))
    return r


def uniform_ints(n, lo, hi, seed, salt=0):
    lib = _load()
    out = np.zeros(n, dtype=np.int64)
    lib.synth_uniform_ints(n, lo, hi, ctypes.c_uint64(seed), salt, _ptr(out, ctypes.c_int64))
    return out


# ----------------------------------------------------------------- workloads

def erdos_renyi(N=50, B=20_000, p=0.2, j_exc=0.5, j_inh=-1.5, rate=5.0, tau=0.010,
                dt=0.001, seed=0, f_exc=0.8, name="erdos_renyi") -> Recording:
    """Bernoulli(p) connectivity without self-loops, constant base rate."""
    n_exc = int(round(f_exc * N))
    J = net_bernoulli(N, n_exc, p, j_exc, j_inh, seed)
    mu = np.full(N, math.log(rate))
    bins, neu = simulate(N, B, dt, tau, mu, J, seed)
    return Recording(name, N, B, dt, tau, bins, neu, J, mu, n_exc, seed)


def balanced(N=1000, B=3_600_000, in_frac=0.1, j_exc=0.2, j_inh=-1.0, j_self=-5.0,
             rate_lo=5.0, rate_hi=10.0, tau=0.010, dt=0.001, seed=0, f_exc=0.8,
             name="balanced") -> Recording:
    """Balanced random network with fixed in-degree in_frac*N, split 80/20 E/I,
    base rates c_i ~ U[rate_lo, rate_hi], and an inhibitory self-connection
    j_self modelling refractoriness (Sec. 3.1 uses J_s = 5 J_i; without it the
    exp-link network leaves the 5-10 Hz regime and saturates)."""
    n_exc = int(round(f_exc * N))
    k = int(round(in_frac * N))
    k_exc = int(round(f_exc * k))
    k_inh = k - k_exc
    J = net_fixed_indegree(N, n_exc, k_exc, k_inh, j_exc, j_inh, seed)
    np.fill_diagonal(J, j_self)
    mu = np.log(rates_uniform(N, rate_lo, rate_hi, seed))
    bins, neu = simulate(N, B, dt, tau, mu, J, seed)
    return Recording(name, N, B, dt, tau, bins, neu, J, mu, n_exc, seed)


def synfire(N=1000, B=600_000, p_bg=0.05, j_exc=0.2, j_inh=-1.0, j_self=-20.0,
            n_groups=10, group_size=50, p_chain=0.5, j_chain=0.4, rate_lo=5.0,
            rate_hi=10.0, tau=0.010, dt=0.001, seed=0, f_exc=0.8,
            name="synfire") -> Recording:
    """Synfire chain (n_groups x group_size excitatory neurons) embedded in a
    Bernoulli(p_bg) balanced background, with an inhibitory self-connection
    j_self.  The chain drive (50 x 0.5 x 0.4 per volley) saturates the groups
    unless refractoriness is at least about -20; -5 and -10 both run away."""
    n_exc = int(round(f_exc * N))
    J, g = net_synfire(N, n_exc, p_bg, j_exc, j_inh, n_groups, group_size, p_chain, j_chain,
                       seed)
    np.fill_diagonal(J, j_self)
    mu = np.log(rates_uniform(N, rate_lo, rate_hi, seed))
    bins, neu = simulate(N, B, dt, tau, mu, J, seed)
    return Recording(name, N, B, dt, tau, bins, neu, J, mu, n_exc, seed, group_of=g)


# The five named workloads ------------------------------------------------

def config1(seed=0) -> Recording:
    """N=50 (40E/10I), Bernoulli p=0.2 without self-loops, J_E=+0.5, J_I=-1.5,
    5 Hz base rate, tau=10 ms, dt=1 ms, T=20 s (2e4 bins)."""
    return erdos_renyi(N=50, B=20_000, p=0.2, j_exc=0.5, j_inh=-1.5, rate=5.0, tau=0.010,
                       dt=0.001, seed=seed, name="er_n50_t20s")


def config2(seed=0, B=3_600_000) -> Recording:
    """N=1000 (800E/200I) balanced network, fixed in-degree 100 (80E+20I),
    J_E=+0.2, J_I=-1.0, c_i ~ U[5,10] Hz, tau=10 ms, dt=1 ms, T=3600 s."""
    return balanced(N=1000, B=B, seed=seed, name=f"balanced_n1000_b{B}")


def config4(seed=0, B=600_000) -> Recording:
    """Config-2 generator at N=500 (in-degree 50), T=600 s, true tau=8 ms."""
    return balanced(N=500, B=B, tau=0.008, seed=seed, name=f"balanced_n500_b{B}_tau8ms")


def config5_sizes(n_rec=64, base_seed=1000):
    """(kind, N, B) per recording r: even r balanced, odd r synfire.
    N ~ U{100..2000} (synfire: U{625..2000} so that 10x50 excitatory neurons
    fit), T ~ U[60, 600] s in whole ms."""
    out = []
    for r in range(n_rec):
        seed = base_seed + r
        kind = "balanced" if r % 2 == 0 else "synfire"
        lo = 100 if kind == "balanced" else 625
        N = int(uniform_ints(1, lo, 2000, seed, salt=1)[0])
        B = int(uniform_ints(1, 60_000, 600_000, seed, salt=2)[0])
        out.append((kind, N, B, seed))
    return out


def config5_recording(kind, N, B, seed) -> Recording:
    if kind == "balanced":
        return balanced(N=N, B=B, seed=seed, name=f"balanced_n{N}_b{B}")
    return synfire(N=N, B=B, seed=seed, name=f"synfire_n{N}_b{B}")


# ------------------------------------------------------------------ cache

CACHE_VERSION = 1


def cached(name: str, **kw) -> Recording:
    """Call workload function `name` (e.g. "config2") with kw, memoised on disk
    under $SYNTH_CACHE_DIR (default /tmp/synth_cache) so that several
    processes of one session share a generated raster."""
    import json
    import hashlib
    d = os.environ.get("SYNTH_CACHE_DIR", "/tmp/synth_cache")
    key = hashlib.sha1(json.dumps([CACHE_VERSION, name, sorted(kw.items())],
                                  default=str).encode()).hexdigest()[:16]
    path = os.path.join(d, f"{name}_{key}.npz")
    if os.path.exists(path):
        z = np.load(path, allow_pickle=False)
        meta = json.loads(str(z["meta"]))
        return Recording(meta["name"], meta["n_neurons"], meta["n_bins"], meta["dt"], meta["tau"],
                         z["bins"], z["neurons"], z["J"], z["mu"], meta["n_exc"], meta["seed"],
                         z["group_of"] if "group_of" in z.files else None)
    rec = globals()[name](**kw)
    os.makedirs(d, exist_ok=True)
    meta = dict(name=rec.name, n_neurons=rec.n_neurons, n_bins=rec.n_bins, dt=rec.dt, tau=rec.tau,
                n_exc=rec.n_exc, seed=rec.seed)
    extra = {"group_of": rec.group_of} if rec.group_of is not None else {}
    tmp = path + f".{os.getpid()}.tmp.npz"
    np.savez(tmp, bins=rec.bins, neurons=rec.neurons, J=rec.J, mu=rec.mu,
             meta=np.array(json.dumps(meta)), **extra)
    os.replace(tmp, path)
    return rec
