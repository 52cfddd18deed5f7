"""ctypes wrapper of the FP64 CPU oracle (kgdb_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
benchmark's CPU-baseline leg.  The GPU product path never imports this module.
"""
import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "kgdb_oracle.c")
_LIB = os.path.join(_HERE, "libkgdb_oracle.so")

STREAM_WALK, STREAM_VEL, STREAM_LANGEVIN, STREAM_DB, STREAM_WARMUP = 1, 2, 3, 4, 5
TF_PHANTOM, TF_NOFORCE = 1, 2


def build(force=False):
    """Compile the oracle with gcc (plain -O2, no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-O2", "-std=gnu11", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
               "-shared", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class Params(C.Structure):
    _fields_ = [
        ("M", C.c_int32), ("N", C.c_int32),
        ("rho", C.c_double), ("kappa", C.c_double), ("n_exp", C.c_double),
        ("k_fene", C.c_double), ("R0", C.c_double), ("T", C.c_double),
        ("gamma", C.c_double), ("dt", C.c_double), ("db_rmax", C.c_double),
        ("db_rate", C.c_double),
        ("proposal", C.c_int32), ("precision", C.c_int32),
        ("warmup_steps", C.c_int32),
        ("warmup_dt0", C.c_double), ("warmup_max_disp", C.c_double),
        ("warmup_fcap", C.c_double), ("fene_floor", C.c_double),
        ("seed", C.c_uint64), ("melt_id", C.c_int32), ("test_flags", C.c_uint32),
        ("r_cell", C.c_double),
        ("init_mode", C.c_int32), ("init_tries", C.c_int32), ("init_tol", C.c_double),
    ]


class Stats(C.Structure):
    _fields_ = [
        ("attempts", C.c_int64), ("no_candidate", C.c_int64), ("accepted", C.c_int64),
        ("reverse_impossible", C.c_int64), ("sum_ncand", C.c_int64),
        ("sum_dE_accepted", C.c_double), ("ncand_end", C.c_int64),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


DEFAULTS = dict(M=20, N=50, rho=0.85, kappa=1.5, n_exp=2.0, k_fene=0.0, R0=1.5, T=1.0,
                gamma=1.0, dt=0.01, db_rmax=1.3, db_rate=1e-3, proposal=0, precision=0,
                warmup_steps=1000, warmup_dt0=0.001, warmup_max_disp=0.05, warmup_fcap=10.0,
                fene_floor=0.02, seed=1,
                melt_id=0, test_flags=0, r_cell=0.0, init_mode=0, init_tries=0, init_tol=0.0)

_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(_LIB)
        P = C.c_void_p
        dp = np.ctypeslib.ndpointer(np.float64, flags="C")
        ip = np.ctypeslib.ndpointer(np.int32, flags="C")
        up = np.ctypeslib.ndpointer(np.uint64, flags="C")
        L.kgdbref_last_error.restype = C.c_char_p
        L.kgdbref_philox.argtypes = [up, up, up]
        L.kgdbref_normals.argtypes = [C.c_uint64] * 5 + [dp]
        u32p = np.ctypeslib.ndpointer(np.uint32, flags="C")
        L.kgdbref_philox4x32.argtypes = [u32p, u32p, u32p]
        L.kgdbref_md_normals.argtypes = [C.c_uint64] * 5 + [dp]
        for f in ("kgdbref_mie",):
            getattr(L, f).restype = C.c_double
            getattr(L, f).argtypes = [C.c_double] * 3
        for f in ("kgdbref_mlj", "kgdbref_pair_u", "kgdbref_pair_f"):
            getattr(L, f).restype = C.c_double
            getattr(L, f).argtypes = [C.c_double] * 2
        L.kgdbref_kn.restype = C.c_double
        L.kgdbref_kn.argtypes = [C.c_double] * 3
        for f in ("kgdbref_fene_u", "kgdbref_fene_f"):
            getattr(L, f).restype = C.c_double
            getattr(L, f).argtypes = [C.c_double] * 4
        L.kgdbref_create.restype = P
        L.kgdbref_create.argtypes = [C.POINTER(Params)]
        L.kgdbref_create_empty.restype = P
        L.kgdbref_create_empty.argtypes = [C.POINTER(Params)]
        L.kgdbref_destroy.argtypes = [P]
        L.kgdbref_box.restype = C.c_double
        L.kgdbref_box.argtypes = [P]
        L.kgdbref_kfene.restype = C.c_double
        L.kgdbref_kfene.argtypes = [P]
        L.kgdbref_get_state.argtypes = [P, P, P, P, P, P, P]
        L.kgdbref_set_state.argtypes = [P, P, P, P, P, P]
        L.kgdbref_forces.argtypes = [P, C.c_int32, P, P, P]
        L.kgdbref_md_steps.argtypes = [P, C.c_int64]
        L.kgdbref_set_potential.argtypes = [P, C.c_double, C.c_double]
        L.kgdbref_init_info.argtypes = [P, dp]
        L.kgdbref_pair_hist.argtypes = [P, C.c_double, C.c_int32, up]
        L.kgdbref_structure_factor.argtypes = [P, ip, C.c_int64, dp]
        L.kgdbref_msd_reset.argtypes = [P]
        L.kgdbref_msd_reset.restype = None
        L.kgdbref_msd.argtypes = [P]
        L.kgdbref_msd.restype = C.c_double
        L.kgdbref_cell_list.argtypes = [P, C.c_double, C.POINTER(C.c_int32), P, P, C.c_int64]
        L.kgdbref_candidates.argtypes = [P, C.c_int32, P, C.c_int64, C.POINTER(C.c_int64)]
        L.kgdbref_db_sweep.argtypes = [P, C.c_int64, C.c_int32, C.POINTER(Stats)]
        L.kgdbref_move_dE.restype = C.c_double
        L.kgdbref_move_dE.argtypes = [P] + [C.c_int32] * 5
        L.kgdbref_apply_move.argtypes = [P] + [C.c_int32] * 5
        L.kgdbref_observables.argtypes = [P, P, P, P]
        L.kgdbref_energy.argtypes = [P, P]
        L.kgdbref_fit_ellK.argtypes = [dp, C.c_int32, C.c_double, C.POINTER(C.c_double)]
        # learned proposal
        L.kgdbref_mlp_nparam.restype = C.c_int32
        L.kgdbref_features.argtypes = [P, P, C.c_int64, P]
        L.kgdbref_mlp_forward.argtypes = [P, P, C.c_int64, P]
        L.kgdbref_mlp_quantised.argtypes = [P, P]
        L.kgdbref_mlp_grad.argtypes = [P, P, P, C.c_int64, P, P]
        L.kgdbref_mlp_surrogate_loss.restype = C.c_double
        L.kgdbref_mlp_surrogate_loss.argtypes = [P, P, P, P, C.c_int64]
        L.kgdbref_adam.argtypes = [P, P, P, P, C.c_int64, C.c_double, C.c_double, C.c_double, C.c_double, P, P, P]
        L.kgdbref_learned_q.argtypes = [P, P, C.c_double, P, P, C.c_int64, C.POINTER(C.c_int64)]
        L.kgdbref_db_sweep_learned.argtypes = [P, C.c_int64, P, C.c_double, C.POINTER(Stats)]
        L.kgdbref_db_sweep_log.argtypes = [P, C.c_int64, C.c_int32, C.POINTER(Stats), P, P, C.c_int64,
                                           C.POINTER(C.c_int64)]
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _check(rc):
    if rc != 0:
        raise RuntimeError(f"oracle error {rc}: {lib().kgdbref_last_error().decode()}")


def philox(ctr, key):
    out = np.zeros(4, np.uint64)
    lib().kgdbref_philox(np.asarray(ctr, np.uint64), np.asarray(key, np.uint64), out)
    return out


def normals(seed, melt, i_lo, i_hi, stream):
    z = np.zeros(4)
    lib().kgdbref_normals(seed, melt, i_lo, i_hi, stream, z)
    return z


def philox4x32(ctr, key):
    out = np.zeros(4, np.uint32)
    lib().kgdbref_philox4x32(np.asarray(ctr, np.uint32), np.asarray(key, np.uint32), out)
    return out


def md_normals(seed, melt, i, t, stream):
    """The four normals of the MD kick of monomer i at step t (Philox4x32-10)."""
    z = np.zeros(4)
    lib().kgdbref_md_normals(seed, melt, i, t, stream, z)
    return z


def mie(n, m, r): return lib().kgdbref_mie(n, m, r)
def mlj(n, r): return lib().kgdbref_mlj(n, r)
def pair_u(n, r): return lib().kgdbref_pair_u(n, r)
def pair_f(n, r): return lib().kgdbref_pair_f(n, r)
def kn(n, l0=0.960897, R0=1.5): return lib().kgdbref_kn(n, l0, R0)
def fene_u(k, R0, r, amin=0.0): return lib().kgdbref_fene_u(k, R0, r, amin)
def fene_f(k, R0, r, amin=0.0): return lib().kgdbref_fene_f(k, R0, r, amin)


def fit_ellK(r2n, N, l0):
    out = C.c_double()
    _check(lib().kgdbref_fit_ellK(np.ascontiguousarray(r2n, np.float64), N, l0, C.byref(out)))
    return out.value


def make_params(**kw):
    d = dict(DEFAULTS)
    d.update(kw)
    return Params(**d)


class Melt:
    """One melt held by the oracle."""

    def __init__(self, empty=False, **kw):
        self.p = make_params(**kw)
        L = lib()
        h = (L.kgdbref_create_empty if empty else L.kgdbref_create)(C.byref(self.p))
        if not h:
            raise RuntimeError("oracle init failed: " + L.kgdbref_last_error().decode())
        self.h = h
        self.M, self.N = self.p.M, self.p.N
        self.Nm = self.M * self.N
        self.L = L.kgdbref_box(h)
        self.kfene = L.kgdbref_kfene(h)

    def __del__(self):
        if getattr(self, "h", None):
            lib().kgdbref_destroy(self.h)
            self.h = None

    def get_state(self):
        x = np.zeros((3, self.Nm)); v = np.zeros((3, self.Nm))
        fc = np.zeros((3, self.Nm)); fl = np.zeros((3, self.Nm))
        ch = np.zeros(self.Nm, np.int32); cnt = np.zeros(4, np.uint64)
        _check(lib().kgdbref_get_state(self.h, _ptr(x), _ptr(v), _ptr(fc), _ptr(fl), _ptr(ch), _ptr(cnt)))
        return dict(x=x, v=v, fc=fc, fl=fl, chains=ch.reshape(self.M, self.N), counters=cnt)

    def set_state(self, x=None, v=None, fl=None, chains=None, counters=None):
        cv = lambda a, t: None if a is None else np.ascontiguousarray(a, t)
        x, v, fl = cv(x, np.float64), cv(v, np.float64), cv(fl, np.float64)
        ch, cnt = cv(chains, np.int32), cv(counters, np.uint64)
        _check(lib().kgdbref_set_state(self.h, _ptr(x), _ptr(v), _ptr(fl), _ptr(ch), _ptr(cnt)))

    def forces(self, brute=False):
        F = np.zeros((3, self.Nm)); S = np.zeros(self.Nm); E = np.zeros(3)
        _check(lib().kgdbref_forces(self.h, int(brute), _ptr(F), _ptr(S), _ptr(E)))
        return F, S, E

    def md_steps(self, n):
        _check(lib().kgdbref_md_steps(self.h, n))

    def pair_hist(self, r_max, nbins):
        """Ordered-pair counts of minimum-image distances in nbins bins over [0, r_max)."""
        out = np.zeros(nbins, np.uint64)
        _check(lib().kgdbref_pair_hist(self.h, float(r_max), int(nbins), out))
        return out

    def structure_factor(self, nvec):
        """S(q) for reciprocal-lattice vectors q = 2 pi n / L (n: [nq][3] integers)."""
        n = np.ascontiguousarray(nvec, np.int32).reshape(-1, 3)
        out = np.zeros(len(n))
        _check(lib().kgdbref_structure_factor(self.h, n.ravel(), len(n), out))
        return out

    def msd_reset(self):
        lib().kgdbref_msd_reset(self.h)

    def msd(self):
        return lib().kgdbref_msd(self.h)

    def init_info(self):
        """(init mode, states drawn, l_K fitted to the accepted freely rotating state)."""
        out = np.zeros(3)
        _check(lib().kgdbref_init_info(self.h, out))
        return int(out[0]), int(out[1]), out[2]

    def set_potential(self, n_exp, k_fene=0.0):
        _check(lib().kgdbref_set_potential(self.h, float(n_exp), float(k_fene)))

    def cell_list(self, rcell=0.0):
        nc = C.c_int32()
        _check(lib().kgdbref_cell_list(self.h, rcell, C.byref(nc), None, None, 0))
        start = np.zeros(nc.value ** 3 + 1, np.int32); srt = np.zeros(self.Nm, np.int32)
        _check(lib().kgdbref_cell_list(self.h, rcell, C.byref(nc), _ptr(start), _ptr(srt), start.size))
        return nc.value, start, srt

    def candidates(self, brute=False, cap=1 << 20):
        keys = np.zeros(cap, np.uint64); n = C.c_int64()
        _check(lib().kgdbref_candidates(self.h, int(brute), _ptr(keys), cap, C.byref(n)))
        return keys[: n.value].copy()

    def db_sweep(self, K, brute=False):
        st = Stats()
        _check(lib().kgdbref_db_sweep(self.h, K, int(brute), C.byref(st)))
        return st.as_dict()

    def move_dE(self, A, i, B, j, var):
        return lib().kgdbref_move_dE(self.h, A, i, B, j, var)

    def apply_move(self, A, i, B, j, var):
        _check(lib().kgdbref_apply_move(self.h, A, i, B, j, var))

    def db_sweep_log(self, K, cap=1 << 16, brute=False):
        """Uniform sweep that records (inputs, accepted) of every attempt with candidates."""
        st = Stats()
        feat = np.zeros((cap, NN_IN), np.float32); lab = np.zeros(cap, np.int32); n = C.c_int64()
        _check(lib().kgdbref_db_sweep_log(self.h, K, int(brute), C.byref(st), _ptr(feat), _ptr(lab), cap, C.byref(n)))
        return st.as_dict(), feat[: n.value].copy(), lab[: n.value].copy()

    def db_sweep_learned(self, K, params, mix):
        st = Stats()
        P = np.ascontiguousarray(params, np.float32)
        _check(lib().kgdbref_db_sweep_learned(self.h, K, _ptr(P), float(mix), C.byref(st)))
        return st.as_dict()

    def features(self, keys):
        keys = np.ascontiguousarray(keys, np.uint64)
        out = np.zeros((keys.size, NN_IN), np.float32)
        _check(lib().kgdbref_features(self.h, _ptr(keys), keys.size, _ptr(out)))
        return out

    def learned_q(self, params, mix, cap=1 << 16):
        keys = np.zeros(cap, np.uint64); q = np.zeros(cap); n = C.c_int64()
        P = np.ascontiguousarray(params, np.float32)
        _check(lib().kgdbref_learned_q(self.h, _ptr(P), float(mix), _ptr(keys), _ptr(q), cap, C.byref(n)))
        return keys[: n.value].copy(), q[: n.value].copy()

    def observables(self):
        r2n = np.zeros(self.N - 1); lk = C.c_double(); mb = C.c_double()
        _check(lib().kgdbref_observables(self.h, _ptr(r2n), C.byref(lk), C.byref(mb)))
        return r2n, lk.value, mb.value

    def energy(self):
        e = np.zeros(4)
        _check(lib().kgdbref_energy(self.h, _ptr(e)))
        return e


def key_decode(key, M, N):
    """(A, i, B, j, variant) of a candidate key; i, j are 1-based bond indices."""
    key = int(key)
    Nb = N - 1
    var = key & 1
    q = key >> 1
    hi, lo = divmod(q, M * Nb)
    return hi // Nb, hi % Nb + 1, lo // Nb, lo % Nb + 1, var


# ---------------------------------------------------------------- learned proposal network
NN_IN, NN_H = 25, 128
NN_NPARAM = NN_H * NN_IN + NN_H + 2 * (NN_H * NN_H + NN_H) + NN_H + 1


def nn_slices():
    """Offsets of W1 [128][25], b1, W2 [128][128], b2, W3, b3, w4 [128], b4 in the parameter vector."""
    sl, o = {}, 0
    for name, size in (("W1", NN_H * NN_IN), ("b1", NN_H), ("W2", NN_H * NN_H), ("b2", NN_H),
                       ("W3", NN_H * NN_H), ("b3", NN_H), ("w4", NN_H), ("b4", 1)):
        sl[name] = slice(o, o + size)
        o += size
    assert o == NN_NPARAM
    return sl


def mlp_forward(params, x):
    P = np.ascontiguousarray(params, np.float32)
    x = np.ascontiguousarray(x, np.float32).reshape(-1, NN_IN)
    out = np.zeros(x.shape[0], np.float32)
    _check(lib().kgdbref_mlp_forward(_ptr(P), _ptr(x), x.shape[0], _ptr(out)))
    return out


def mlp_quantised(params):
    P = np.ascontiguousarray(params, np.float32)
    out = np.zeros(NN_NPARAM)
    lib().kgdbref_mlp_quantised(_ptr(P), _ptr(out))
    return out


def mlp_grad(params, x, y):
    P = np.ascontiguousarray(params, np.float32)
    x = np.ascontiguousarray(x, np.float32).reshape(-1, NN_IN)
    y = np.ascontiguousarray(y, np.int32)
    g = np.zeros(NN_NPARAM); loss = np.zeros(1)
    _check(lib().kgdbref_mlp_grad(_ptr(P), _ptr(x), _ptr(y), x.shape[0], _ptr(g), _ptr(loss)))
    return g, float(loss[0])


def mlp_surrogate_loss(params0, params, x, y):
    P0 = np.ascontiguousarray(params0, np.float32)
    Pd = np.ascontiguousarray(params, np.float64)
    x = np.ascontiguousarray(x, np.float32).reshape(-1, NN_IN)
    y = np.ascontiguousarray(y, np.int32)
    return lib().kgdbref_mlp_surrogate_loss(_ptr(P0), _ptr(Pd), _ptr(x), _ptr(y), x.shape[0])


def adam(params, m, v, g, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    P = np.ascontiguousarray(params, np.float32)
    m = np.ascontiguousarray(m, np.float32); v = np.ascontiguousarray(v, np.float32)
    g = np.ascontiguousarray(g, np.float64)
    Po, mo, vo = np.zeros(NN_NPARAM), np.zeros(NN_NPARAM), np.zeros(NN_NPARAM)
    lib().kgdbref_adam(_ptr(P), _ptr(m), _ptr(v), _ptr(g), t, lr, b1, b2, eps, _ptr(Po), _ptr(mo), _ptr(vo))
    return Po, mo, vo
