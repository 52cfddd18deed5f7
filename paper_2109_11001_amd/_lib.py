"""ctypes binding of libkgdb.so (the HIP C ABI declared in include/kgdb.h).

Argument marshalling only: every step of the hot path runs in the library's kernels.
Loading fails loudly when the library has not been built.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libkgdb.so")

E_PARAM, E_ALLOC, E_HIP, E_FENE, E_NONFINITE, E_OVERFLOW, E_STATE = -1, -2, -3, -4, -5, -6, -7
PROPOSAL_UNIFORM, PROPOSAL_LEARNED, PROPOSAL_LITERAL = 0, 1, 2
PREC_FP64, PREC_MIXED = 0, 1
INIT_RANDOM_WALK, INIT_FREELY_ROTATING = 0, 1
TF_PHANTOM, TF_NOFORCE, TF_NL_GLOBAL, TF_SIDE_FAULT, TF_DB_GLOBAL = 1, 2, 4, 8, 16


class KgdbError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"kgdb error {code}: {msg}")
        self.code = code


class Params(C.Structure):
    _fields_ = [
        ("M", C.c_int32), ("N", C.c_int32),
        ("rho", C.c_double), ("kappa", C.c_double), ("n_exp", C.c_double),
        ("k_fene", C.c_double), ("R0", C.c_double),
        ("T", C.c_double), ("gamma", C.c_double), ("dt", C.c_double),
        ("db_rmax", C.c_double), ("db_rate", C.c_double),
        ("proposal", C.c_int32), ("precision", C.c_int32), ("warmup_steps", C.c_int32),
        ("warmup_dt0", C.c_double), ("warmup_max_disp", C.c_double), ("warmup_fcap", C.c_double),
        ("fene_floor", C.c_double),
        ("seed", C.c_uint64), ("melt_id", C.c_int32), ("test_flags", C.c_uint32),
        ("r_cell", C.c_double), ("nl_every", C.c_int32), ("nl_skin", C.c_double),
        ("init_mode", C.c_int32), ("init_tries", C.c_int32), ("init_tol", C.c_double),
    ]


class DbStats(C.Structure):
    _fields_ = [
        ("attempts", C.c_int64), ("no_candidate", C.c_int64), ("accepted", C.c_int64),
        ("reverse_impossible", C.c_int64), ("sum_ncand", C.c_int64),
        ("sum_dE_accepted", C.c_double), ("ncand_end", C.c_int64),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class StageStats(C.Structure):
    _fields_ = [
        ("n_exp", C.c_double), ("steps", C.c_int64), ("attempts", C.c_int64), ("no_candidate", C.c_int64),
        ("accepted", C.c_int64), ("wall_ms", C.c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


# every symbol include/kgdb.h declares
EXPORTS = [
    "kgdb_init_batch", "kgdb_init_melt", "kgdb_destroy", "kgdb_last_error", "kgdb_batch_size",
    "kgdb_md_steps", "kgdb_db_sweep", "kgdb_observables", "kgdb_energy", "kgdb_get_state",
    "kgdb_set_state", "kgdb_forces", "kgdb_cell_list", "kgdb_candidates", "kgdb_db_probe",
    "kgdb_time_force_kernel", "kgdb_db_sweep_checked", "kgdb_profile", "kgdb_profile_read",
    "kgdb_melt_geometry", "kgdb_batch_sizes", "kgdb_autotune", "kgdb_nl_info",
    "kgdb_mlp_nparam", "kgdb_set_proposal_net", "kgdb_db_sweep_log", "kgdb_features", "kgdb_candidate_logits",
    "kgdb_mlp_workspace_bytes", "kgdb_mlp_forward", "kgdb_mlp_grad", "kgdb_mlp_adam", "kgdb_mlp_train_step",
    "kgdb_set_potential", "kgdb_protocol_schedule", "kgdb_run_protocol", "kgdb_init_info",
    "kgdb_pair_correlation", "kgdb_structure_factor", "kgdb_msd_reset", "kgdb_msd",
    "kgdb_mlp_train_step_static", "kgdb_fene_floored", "kgdb_nl_stats", "kgdb_tile_shapes", "kgdb_set_tiles",
]
MLP_STATIC_ROWS = 4096
MLP_NPARAM = 36481

_lib = None


def load():
    """Load libkgdb.so (built in-tree by paper_2109_11001_amd/build.py)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2109_11001_amd.build` "
                          "(or __graft_entry__.build()); there is no fallback path")
    L = C.CDLL(LIB_PATH)
    P = C.c_void_p
    i32, i64, dbl = C.c_int32, C.c_int64, C.c_double
    L.kgdb_last_error.restype = C.c_char_p
    L.kgdb_init_batch.argtypes = [C.POINTER(Params), i32, P, C.POINTER(P)]
    L.kgdb_init_melt.argtypes = [C.POINTER(Params), P, C.POINTER(P)]
    L.kgdb_destroy.argtypes = [P]
    L.kgdb_destroy.restype = None
    L.kgdb_batch_size.argtypes = [P]
    L.kgdb_batch_size.restype = i32
    L.kgdb_md_steps.argtypes = [P, i64, i32]
    L.kgdb_db_sweep.argtypes = [P, i64, P]
    L.kgdb_db_sweep_checked.argtypes = [P, i64, P]
    L.kgdb_observables.argtypes = [P, i32, P, P, P]
    L.kgdb_energy.argtypes = [P, i32, P]
    L.kgdb_get_state.argtypes = [P, i32, P, P, P, P, P, P]
    L.kgdb_set_state.argtypes = [P, i32, P, P, P, P, P]
    L.kgdb_forces.argtypes = [P, i32, P, P, P]
    L.kgdb_cell_list.argtypes = [P, i32, P, P, P, i64]
    L.kgdb_candidates.argtypes = [P, i32, P, i64, P]
    L.kgdb_db_probe.argtypes = [P, i32, P, i64, P, P]
    L.kgdb_time_force_kernel.argtypes = [P, i32, P]
    L.kgdb_profile.argtypes = [P, i32]
    L.kgdb_profile_read.argtypes = [P, P, P, P, P]
    L.kgdb_melt_geometry.argtypes = [P, i32, P]
    L.kgdb_batch_sizes.argtypes = [P, P, P]
    L.kgdb_autotune.argtypes = [P, i32, i32, P, P]
    L.kgdb_nl_info.argtypes = [P, P]
    L.kgdb_fene_floored.argtypes = [P, i32, P]
    L.kgdb_nl_stats.argtypes = [P, P]
    L.kgdb_tile_shapes.argtypes = [P, P]
    L.kgdb_set_tiles.argtypes = [P, i32, i32]
    L.kgdb_mlp_nparam.argtypes = []
    L.kgdb_set_proposal_net.argtypes = [P, P, i32, dbl]
    L.kgdb_db_sweep_log.argtypes = [P, i64, P, P, P, i64, P]
    L.kgdb_features.argtypes = [P, i32, P, i64, P]
    L.kgdb_candidate_logits.argtypes = [P, i32, P, P, i64, P]
    L.kgdb_mlp_workspace_bytes.argtypes = [i64]
    L.kgdb_mlp_forward.argtypes = [P, P, i64, P, P, i64, P]
    L.kgdb_mlp_grad.argtypes = [P, P, P, i64, P, P, P, i64, P]
    L.kgdb_mlp_adam.argtypes = [P, P, P, P, i64, dbl, dbl, dbl, dbl, P]
    L.kgdb_mlp_train_step.argtypes = [P, P, P, P, P, i64, i64, dbl, dbl, dbl, dbl, P, i64, P, P]
    L.kgdb_mlp_train_step_static.argtypes = [P, P, P, P, P, i64, i64, dbl, dbl, dbl, dbl, P, P]
    L.kgdb_set_potential.argtypes = [P, i32, dbl, dbl]
    L.kgdb_init_info.argtypes = [P, i32, P]
    L.kgdb_pair_correlation.argtypes = [P, i32, dbl, i32, P, P]
    L.kgdb_structure_factor.argtypes = [P, i32, P, i64, P]
    L.kgdb_msd_reset.argtypes = [P]
    L.kgdb_msd.argtypes = [P, i32, P]
    L.kgdb_protocol_schedule.argtypes = [dbl, i32, dbl, dbl, P, P, P]
    L.kgdb_run_protocol.argtypes = [P, P, P, i32, i64, P]
    for f in EXPORTS:
        if f not in ("kgdb_destroy", "kgdb_last_error", "kgdb_batch_size"):
            getattr(L, f).restype = C.c_int
    L.kgdb_mlp_nparam.restype = i64
    L.kgdb_mlp_workspace_bytes.restype = i64
    _lib = L
    return L


def check(rc):
    if rc != 0:
        raise KgdbError(rc, load().kgdb_last_error().decode())


def ptr(a):
    return None if a is None else C.c_void_p(a.ctypes.data)
