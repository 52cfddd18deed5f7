"""kgdb: MI355X-native Langevin MD of semiflexible Kremer-Grest melts under the core-softened
MLJ^n potential, interleaved with double-bridging Monte Carlo (Dietz & Hoy, arXiv 2109.11001).

The Python layer only marshals arguments to the HIP C ABI of libkgdb.so; PyTorch may supply
the HIP stream.
"""
import ctypes as C

import numpy as np

from ._lib import (PREC_FP64, PREC_MIXED, PROPOSAL_LITERAL, PROPOSAL_UNIFORM, TF_NL_GLOBAL, TF_NOFORCE,
                   TF_PHANTOM, DbStats, KgdbError, Params, check, load, ptr)

DEFAULTS = dict(M=20, N=50, rho=0.85, kappa=1.5, n_exp=2.0, k_fene=0.0, R0=1.5, T=1.0,
                gamma=1.0, dt=0.01, db_rmax=1.3, db_rate=1e-3, proposal=PROPOSAL_UNIFORM,
                precision=PREC_FP64, warmup_steps=1000, warmup_dt0=0.001, warmup_max_disp=0.05,
                warmup_fcap=10.0, fene_floor=0.02, seed=1, melt_id=0, test_flags=0, r_cell=0.0,
                nl_every=0, nl_skin=0.0)

# the n values of the paper's schedule, Eq. (11)
XI = (2.0, 3.0, 4.0, 5.0, 5.75, 6.5, 7.0, 8.0, 9.0, 10.0, 11.0, 12.0)


def make_params(**kw):
    d = dict(DEFAULTS)
    unknown = set(kw) - set(d)
    if unknown:
        raise TypeError(f"unknown parameters {sorted(unknown)}")
    d.update(kw)
    return Params(**d)


def _stream_handle(stream):
    if stream is None:
        return None
    h = getattr(stream, "cuda_stream", stream)
    return C.c_void_p(int(h)) if h else None


class Batch:
    """A batch of independent melts advanced together on one GPU."""

    def __init__(self, melts, stream=None):
        if isinstance(melts, dict):
            melts = [melts]
        L = load()
        arr = (Params * len(melts))(*[make_params(**m) for m in melts])
        h = C.c_void_p()
        check(L.kgdb_init_batch(arr, len(melts), _stream_handle(stream), C.byref(h)))
        self._h = h
        self.params = [dict(DEFAULTS, **m) for m in melts]
        self.nm = len(melts)
        self.geom = []
        for k in range(self.nm):
            g = np.zeros(4)
            check(L.kgdb_melt_geometry(h, k, ptr(g)))
            self.geom.append(dict(L=g[0], nc=int(g[1]), nc13=int(g[2]), k_fene=g[3]))

    def close(self):
        h = getattr(self, "_h", None)
        if h:
            self._h = None
            try:
                load().kgdb_destroy(h)
            except Exception:  # interpreter shutdown
                pass

    def __del__(self):
        self.close()

    def _MN(self, k):
        return self.params[k]["M"], self.params[k]["N"]

    def md_steps(self, n, graph=True):
        check(load().kgdb_md_steps(self._h, int(n), int(bool(graph))))

    def db_sweep(self, n_attempts=-1, checked=False):
        st = (DbStats * self.nm)()
        f = load().kgdb_db_sweep_checked if checked else load().kgdb_db_sweep
        check(f(self._h, int(n_attempts), st))
        return [s.as_dict() for s in st]

    def observables(self, melt=0):
        M, N = self._MN(melt)
        r2n = np.zeros(N - 1); lk = C.c_double(); mb = C.c_double()
        check(load().kgdb_observables(self._h, melt, ptr(r2n), C.byref(lk), C.byref(mb)))
        return r2n, lk.value, mb.value

    def energy(self, melt=0):
        e = np.zeros(4)
        check(load().kgdb_energy(self._h, melt, ptr(e)))
        return e

    def get_state(self, melt=0):
        M, N = self._MN(melt)
        Nm = M * N
        x, v, fc, fl = (np.zeros((3, Nm)) for _ in range(4))
        ch = np.zeros(Nm, np.int32); cnt = np.zeros(4, np.uint64)
        check(load().kgdb_get_state(self._h, melt, ptr(x), ptr(v), ptr(fc), ptr(fl), ptr(ch), ptr(cnt)))
        return dict(x=x, v=v, fc=fc, fl=fl, chains=ch.reshape(M, N), counters=cnt)

    def set_state(self, melt=0, x=None, v=None, fl=None, chains=None, counters=None):
        cv = lambda a, t: None if a is None else np.ascontiguousarray(a, t)
        x, v, fl = cv(x, np.float64), cv(v, np.float64), cv(fl, np.float64)
        ch, cnt = cv(chains, np.int32), cv(counters, np.uint64)
        check(load().kgdb_set_state(self._h, melt, ptr(x), ptr(v), ptr(fl), ptr(ch), ptr(cnt)))

    def forces(self, melt=0):
        M, N = self._MN(melt)
        F = np.zeros((3, M * N)); S = np.zeros(M * N); E = np.zeros(3)
        check(load().kgdb_forces(self._h, melt, ptr(F), ptr(S), ptr(E)))
        return F, S, E

    def cell_list(self, melt=0):
        M, N = self._MN(melt)
        nc = C.c_int32()
        check(load().kgdb_cell_list(self._h, melt, C.byref(nc), None, None, 0))
        start = np.zeros(nc.value ** 3 + 1, np.int32); srt = np.zeros(M * N, np.int32)
        check(load().kgdb_cell_list(self._h, melt, C.byref(nc), ptr(start), ptr(srt), start.size))
        return nc.value, start, srt

    def candidates(self, melt=0):
        n = C.c_int64()
        check(load().kgdb_candidates(self._h, melt, None, 0, C.byref(n)))
        keys = np.zeros(max(n.value, 1), np.uint64)
        check(load().kgdb_candidates(self._h, melt, ptr(keys), keys.size, C.byref(n)))
        return keys[: n.value].copy()

    def db_probe(self, keys, melt=0):
        keys = np.ascontiguousarray(keys, np.uint64)
        dE = np.zeros(len(keys)); na = np.zeros(len(keys), np.int64)
        check(load().kgdb_db_probe(self._h, melt, ptr(keys), len(keys), ptr(dE), ptr(na)))
        return dE, na

    def time_force_kernel(self, reps=50):
        ms = C.c_double()
        check(load().kgdb_time_force_kernel(self._h, int(reps), C.byref(ms)))
        return ms.value

    def profile(self, enable=True):
        check(load().kgdb_profile(self._h, int(bool(enable))))

    def profile_read(self):
        fm, fn, nm_, nn = C.c_double(), C.c_int64(), C.c_double(), C.c_int64()
        check(load().kgdb_profile_read(self._h, C.byref(fm), C.byref(fn), C.byref(nm_), C.byref(nn)))
        return dict(force_ms=fm.value, force_n=fn.value, finalize_ms=nm_.value, finalize_n=nn.value)

    def autotune(self, nl_every=0, reps=20):
        """Pick (0) or set the neighbour-list rebuild interval; returns (K, ms per step for K=1,2,5)."""
        ch = C.c_int32(); ms = np.zeros(3)
        check(load().kgdb_autotune(self._h, int(nl_every), int(reps), C.byref(ch), ptr(ms)))
        return ch.value, dict(zip((1, 2, 5), ms))

    def nl_info(self):
        out = np.zeros(4)
        check(load().kgdb_nl_info(self._h, ptr(out)))
        return dict(K=int(out[0]), skin=out[1], mean_list=out[2], rollbacks=int(out[3]))

    def sizes(self):
        a, b = C.c_int64(), C.c_int64()
        check(load().kgdb_batch_sizes(self._h, C.byref(a), C.byref(b)))
        return a.value, b.value


def Melt(stream=None, **kw):
    """A batch holding a single melt."""
    return Batch([kw], stream=stream)
