"""kgdb: MI355X-native Langevin MD of semiflexible Kremer-Grest melts under the core-softened
MLJ^n potential, interleaved with double-bridging Monte Carlo (Dietz & Hoy, arXiv 2109.11001).

The Python layer only marshals arguments to the HIP C ABI of libkgdb.so; PyTorch may supply
the HIP stream.
"""
import ctypes as C

import numpy as np

from ._lib import (INIT_FREELY_ROTATING, INIT_RANDOM_WALK, MLP_NPARAM, PREC_FP64, PREC_MIXED, PROPOSAL_LEARNED,
                   PROPOSAL_LITERAL, PROPOSAL_UNIFORM, TF_DB_GLOBAL, TF_NL_GLOBAL, TF_NOFORCE, TF_PHANTOM, TF_SIDE_FAULT, DbStats, KgdbError,
                   Params, StageStats, check, load, ptr)

NN_IN = 25

DEFAULTS = dict(M=20, N=50, rho=0.85, kappa=1.5, n_exp=2.0, k_fene=0.0, R0=1.5, T=1.0,
                gamma=1.0, dt=0.01, db_rmax=1.3, db_rate=1e-3, proposal=PROPOSAL_UNIFORM,
                precision=PREC_FP64, warmup_steps=1000, warmup_dt0=0.001, warmup_max_disp=0.05,
                warmup_fcap=10.0, fene_floor=0.02, seed=1, melt_id=0, test_flags=0, r_cell=0.0,
                nl_every=0, nl_skin=0.0, init_mode=INIT_RANDOM_WALK, init_tries=0, init_tol=0.0)

# the n values of the paper's schedule, Eq. (11)
XI = (2.0, 3.0, 4.0, 5.0, 5.75, 6.5, 7.0, 8.0, 9.0, 10.0, 11.0, 12.0)
# the prefactor of Eq. (16) that brings the kappa = 5.5, N = 400 run to 10^8 steps of 0.008 tau
F0 = 46.3354


def protocol_schedule(kappa, N, dt=0.01, f=F0):
    """Stage plan of the n-ramp protocol (Sec. II.B, Eqs. 11-12, 16-20), from the library:
    dict(n=[12 exponents], steps=[12 step counts], tau_fix, tau_e, tau_eq, scheme)."""
    n = np.zeros(12)
    steps = np.zeros(12, np.int64)
    taus = np.zeros(4)
    rc = load().kgdb_protocol_schedule(float(kappa), int(N), float(dt), float(f), ptr(n), ptr(steps), ptr(taus))
    if rc < 0:
        raise KgdbError(rc, "invalid schedule arguments")
    return dict(n=n[:rc].tolist(), steps=steps[:rc].tolist(), tau_fix=taus[0], tau_e=taus[1], tau_eq=taus[2],
                scheme=int(taus[3]))


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
        self._stream = stream
        self.params = [dict(DEFAULTS, **m) for m in melts]
        self.nm = len(melts)
        self._read_geometry()

    def _read_geometry(self):
        self.geom = []
        for k in range(self.nm):
            g = np.zeros(4)
            check(load().kgdb_melt_geometry(self._h, k, ptr(g)))
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

    def counters(self, melt=0):
        """{step, sweep, last_sweep_step, fc_valid} of melt `melt` (no state transfer)."""
        cnt = np.zeros(4, np.uint64)
        check(load().kgdb_get_state(self._h, melt, None, None, None, None, None, ptr(cnt)))
        return [int(c) for c in cnt]

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

    def nl_stats(self):
        """LDS stages of the list tiles: tiles read from global memory so far, largest stage,
        current capacity, capacity limit."""
        out = np.zeros(8, np.int64)
        check(load().kgdb_nl_stats(self._h, ptr(out)))
        nm, _ = self.sizes()
        return dict(stage_overflows=int(out[0]), largest_stage=int(out[1]), stage_cap=int(out[2]),
                    stage_cap_max=int(out[3]), staged_per_monomer=float(out[4]) / max(nm, 1), tiles=int(out[5]),
                    tile_shape=(int(out[6]), int(out[7])))

    def tile_shapes(self):
        """Candidate (S, Sy) list-tile shapes of melt 0 at the current rebuild interval."""
        out = np.zeros(6, np.int32)
        check(load().kgdb_tile_shapes(self._h, ptr(out)))
        return [(int(out[2 * c]), int(out[2 * c + 1])) for c in range(3) if out[2 * c] > 0]

    def set_tiles(self, S, Sy):
        """List tiles of S x Sy cells at the current rebuild interval (results unchanged)."""
        check(load().kgdb_set_tiles(self._h, int(S), int(Sy)))

    def fene_floored(self, melt=0):
        """Bond-steps of melt `melt` on the floored FENE continuation (argument below fene_floor)."""
        out = np.zeros(1, np.uint64)
        check(load().kgdb_fene_floored(self._h, int(melt), ptr(out)))
        return int(out[0])

    # ---- structure observables
    def pair_correlation(self, r_max, nbins, melt=0):
        """(ordered-pair counts, g(r)) in nbins bins over [0, r_max)."""
        counts = np.zeros(nbins, np.uint64)
        g = np.zeros(nbins)
        check(load().kgdb_pair_correlation(self._h, int(melt), float(r_max), int(nbins), ptr(counts), ptr(g)))
        return counts, g

    def structure_factor(self, nvec, melt=0):
        """S(q) for reciprocal-lattice vectors q = 2 pi n / L (n: [nq][3] integers)."""
        n = np.ascontiguousarray(nvec, np.int32).reshape(-1, 3)
        out = np.zeros(len(n))
        check(load().kgdb_structure_factor(self._h, int(melt), ptr(n), len(n), ptr(out)))
        return out

    def msd_reset(self):
        check(load().kgdb_msd_reset(self._h))

    def msd(self, melt=0):
        v = C.c_double()
        check(load().kgdb_msd(self._h, int(melt), C.byref(v)))
        return v.value

    def init_info(self, melt=0):
        """(init mode, states drawn, l_K fitted to the accepted freely rotating state)."""
        out = np.zeros(3)
        check(load().kgdb_init_info(self._h, int(melt), ptr(out)))
        return int(out[0]), int(out[1]), out[2]

    def sizes(self):
        a, b = C.c_int64(), C.c_int64()
        check(load().kgdb_batch_sizes(self._h, C.byref(a), C.byref(b)))
        return a.value, b.value

    # ---- n-ramp protocol
    def set_potential(self, n_exp, k_fene=0.0, melt=-1):
        """Exponent n of Eqs. 5-6 and FENE constant (<= 0: Eq. 9) of one melt, or of all (-1)."""
        check(load().kgdb_set_potential(self._h, int(melt), float(n_exp), float(k_fene)))
        for k in ([melt] if melt >= 0 else range(self.nm)):
            self.params[k].update(n_exp=float(n_exp), k_fene=float(k_fene))
        self._read_geometry()

    def run_protocol(self, n_values, steps, sweep_every=100):
        """Run the stages (n_values[i] for steps[i] MD steps, a sweep every sweep_every steps;
        <= 0: no sweeps) in the library; returns one statistics dict per stage."""
        n = np.ascontiguousarray(n_values, np.float64)
        st = np.ascontiguousarray(steps, np.int64)
        if n.shape != st.shape:
            raise ValueError("n_values and steps differ in length")
        out = (StageStats * max(len(n), 1))()
        rc = load().kgdb_run_protocol(self._h, ptr(n), ptr(st), len(n), int(sweep_every), out)
        self._read_geometry()
        check(rc)
        return [out[i].as_dict() for i in range(len(n))]

    # ---- learned proposal
    def set_proposal_net(self, params, mix):
        """Quantise FP32 parameters (numpy array or device tensor) into the batch's network."""
        if hasattr(params, "data_ptr"):
            check(load().kgdb_set_proposal_net(self._h, _dptr(params), 1, float(mix)))
        else:
            p = np.ascontiguousarray(params, np.float32)
            check(load().kgdb_set_proposal_net(self._h, ptr(p), 0, float(mix)))

    def db_sweep_log(self, n_attempts, cap):
        """Uniform sweep recording each attempt: (stats, feat [nm][cap][25], label [nm][cap], n_logged)."""
        import torch
        if self._stream is not None and hasattr(self._stream, "cuda_stream"):
            with torch.cuda.stream(self._stream):  # buffers ordered on the library's stream
                feat = torch.empty((self.nm, cap, NN_IN), dtype=torch.float32, device="cuda")
                lab = torch.empty((self.nm, cap), dtype=torch.int32, device="cuda")
        else:
            feat = torch.empty((self.nm, cap, NN_IN), dtype=torch.float32, device="cuda")
            lab = torch.empty((self.nm, cap), dtype=torch.int32, device="cuda")
            torch.cuda.synchronize()  # the library's own stream is not ordered after torch's
        st = (DbStats * self.nm)()
        nl = np.zeros(self.nm, np.int64)
        check(load().kgdb_db_sweep_log(self._h, int(n_attempts), st, _dptr(feat), _dptr(lab), int(cap), ptr(nl)))
        return [s.as_dict() for s in st], feat, lab, nl

    def features(self, keys, melt=0):
        keys = np.ascontiguousarray(keys, np.uint64)
        out = np.zeros((len(keys), NN_IN), np.float32)
        check(load().kgdb_features(self._h, melt, ptr(keys), len(keys), ptr(out)))
        return out

    def candidate_logits(self, melt=0):
        n = C.c_int64()
        check(load().kgdb_candidate_logits(self._h, melt, None, None, 0, C.byref(n)))
        keys = np.zeros(max(n.value, 1), np.uint64); lg = np.zeros(max(n.value, 1), np.float32)
        check(load().kgdb_candidate_logits(self._h, melt, ptr(keys), ptr(lg), keys.size, C.byref(n)))
        return keys[: n.value].copy(), lg[: n.value].copy()


def Melt(stream=None, **kw):
    """A batch holding a single melt."""
    return Batch([kw], stream=stream)


# ---------------------------------------------------------------- network training (device buffers)
def _dptr(t):
    assert t.is_cuda and t.is_contiguous()
    return C.c_void_p(t.data_ptr())


def _stream_ptr(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(int(s.cuda_stream)) if s.cuda_stream else None


def _workspace(n):
    import torch
    nb = int(load().kgdb_mlp_workspace_bytes(int(n)))
    return torch.empty(nb + 256, dtype=torch.uint8, device="cuda"), nb


def _aligned(ws):
    p = ws.data_ptr()
    return C.c_void_p((p + 255) & ~255)


def mlp_forward(params, feat, stream=None):
    """Logits of input rows feat [n][25] (device tensors)."""
    import torch
    n = feat.shape[0]
    out = torch.empty(n, dtype=torch.float32, device="cuda")
    ws, nb = _workspace(n)
    check(load().kgdb_mlp_forward(_dptr(params), _dptr(feat), n, _dptr(out), _aligned(ws), nb, _stream_ptr(stream)))
    return out


def mlp_grad(params, feat, label, stream=None):
    """(gradient [MLP_NPARAM] float64, mean BCE loss) on device."""
    import torch
    n = feat.shape[0]
    g = torch.empty(MLP_NPARAM, dtype=torch.float64, device="cuda")
    loss = torch.empty(1, dtype=torch.float64, device="cuda")
    ws, nb = _workspace(n)
    check(load().kgdb_mlp_grad(_dptr(params), _dptr(feat), _dptr(label), n, _dptr(g), _dptr(loss), _aligned(ws), nb,
                               _stream_ptr(stream)))
    return g, loss


def mlp_adam(params, m, v, grad, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8, stream=None):
    check(load().kgdb_mlp_adam(_dptr(params), _dptr(m), _dptr(v), _dptr(grad), int(t), lr, b1, b2, eps,
                               _stream_ptr(stream)))


def mlp_train_step_static(params, m, v, feat, label, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8, loss=None,
                          stream=None):
    """One Adam step on device tensors with the library's fixed workspace (no allocation by
    the library; at most MLP_STATIC_ROWS rows).  Returns the loss tensor (device double)."""
    import torch
    n = feat.shape[0]
    if loss is None:
        loss = torch.zeros(1, dtype=torch.float64, device=params.device)
    check(load().kgdb_mlp_train_step_static(_dptr(params), _dptr(m), _dptr(v), _dptr(feat), _dptr(label), n,
                                            int(t), lr, b1, b2, eps, _dptr(loss), _stream_ptr(stream)))
    return loss


class Trainer:
    """FP32 master parameters, Adam moments and a workspace on the device."""

    def __init__(self, params, max_batch, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8, stream=None):
        import torch
        self.params = torch.as_tensor(np.ascontiguousarray(params, np.float32)).cuda()
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.loss = torch.zeros(1, dtype=torch.float64, device="cuda")
        self.ws, self.nb = _workspace(max_batch)
        torch.cuda.synchronize()  # the buffers are used on `stream`
        self.max_batch = max_batch
        self.t = 0
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps
        self.stream = stream

    def step(self, feat, label):
        """One Adam step on a batch (device tensors feat [n][25] float32, label [n] int32)."""
        n = feat.shape[0]
        if n > self.max_batch:
            raise ValueError("batch larger than the workspace")
        self.t += 1
        check(load().kgdb_mlp_train_step(_dptr(self.params), _dptr(self.m), _dptr(self.v), _dptr(feat),
                                         _dptr(label), n, self.t, self.lr, self.b1, self.b2, self.eps,
                                         _aligned(self.ws), self.nb, _dptr(self.loss), _stream_ptr(self.stream)))
        return self.loss
