"""ctypes binding of libpic.so (argument marshalling only).

The structures mirror ``include/pic.h`` field for field.  Every compute step
runs in the HIP library; this module only converts Python values to the C
ABI.  Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpic.so")

PIC_OK, PIC_EINVAL, PIC_ECAPACITY, PIC_EHIP, PIC_ENOCONV, PIC_ENAN, PIC_ESTATE = 0, -1, -2, -3, -4, -5, -6
STATUS_NAMES = {0: "PIC_OK", -1: "PIC_EINVAL", -2: "PIC_ECAPACITY", -3: "PIC_EHIP",
                -4: "PIC_ENOCONV", -5: "PIC_ENAN", -6: "PIC_ESTATE"}

_dp = C.POINTER(C.c_double)
_up = C.POINTER(C.c_uint32)


class PicError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class pic_config(C.Structure):
    _fields_ = [
        ("nr", C.c_int32), ("nz", C.c_int32),
        ("lr", C.c_double), ("lz", C.c_double), ("dt", C.c_double),
        ("scheme", C.c_int32), ("precision", C.c_int32),
        ("cathode_rmax", C.c_double),
        ("circuit", C.c_int32),
        ("v_fixed", C.c_double), ("v_ext", C.c_double), ("r_ext", C.c_double),
        ("gamma_i", C.c_double),
        ("p_gas", C.c_double), ("t_gas", C.c_double),
        ("e_exc", C.c_double), ("e_iz", C.c_double),
        ("sigma", _dp), ("n_table", C.c_int32), ("de_table", C.c_double),
        ("b_r", _dp), ("b_z", _dp),
        ("q", C.c_double * 2), ("m", C.c_double * 2), ("w", C.c_double * 2),
        ("seed", C.c_uint64), ("run", C.c_uint32),
        ("capacity", C.c_int64 * 2),
        ("sort_every", C.c_int32),
        ("poisson_mode", C.c_int32), ("poisson_rtol", C.c_double), ("poisson_maxit", C.c_int32),
        ("wall_bc", C.c_int32 * 3),
        ("frozen_ions", C.c_int32), ("mcc_on", C.c_int32), ("see_on", C.c_int32),
        ("field_solve", C.c_int32),
        ("extra_current", C.c_double),
        ("pc_batch", C.c_int32), ("pc_maxit", C.c_int32),
        ("gamma_e", C.c_double), ("n_meta", C.c_double), ("e_iz_meta", C.c_double),
        ("deposit_fixed", C.c_int32), ("pc_pre", C.c_int32),
    ]


class pic_species_host(C.Structure):
    _fields_ = [("r", _dp), ("z", _dp), ("vr", _dp), ("vt", _dp), ("vz", _dp),
                ("id", _up), ("n", C.c_int64)]


class pic_particle_view(C.Structure):
    _fields_ = [("key_dev", C.c_void_p), ("fr_dev", C.c_void_p), ("fz_dev", C.c_void_p),
                ("vr_dev", C.c_void_p), ("vt_dev", C.c_void_p), ("vz_dev", C.c_void_p),
                ("id_dev", C.c_void_p), ("count", C.c_int64), ("capacity", C.c_int64),
                ("precision", C.c_int32), ("pos_bits", C.c_int32)]


class pic_field_view(C.Structure):
    _fields_ = [("phi_dev", C.c_void_p), ("phi0_dev", C.c_void_p), ("phi_l_dev", C.c_void_p),
                ("q_dev", C.c_void_p * 2), ("nodes", C.c_int64), ("q_precision", C.c_int32),
                ("phi0_prev_dev", C.c_void_p)]


class pic_poisson_stats(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("outer", C.c_int32), ("rel_res", C.c_double),
                ("fell_back", C.c_int32), ("converged", C.c_int32),
                ("pc_iterations", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class pic_diag_out(C.Structure):
    _fields_ = [
        ("step", C.c_int64), ("time", C.c_double),
        ("count", C.c_int64 * 2), ("q_dep", C.c_double * 2), ("q_expect", C.c_double * 2),
        ("ke", C.c_double * 2), ("pz", C.c_double * 2), ("w_field", C.c_double),
        ("dq_conv", C.c_double), ("i_cathode", C.c_double),
        ("vc", C.c_double), ("qc", C.c_double), ("cap_c", C.c_double),
        ("n_peak", C.c_double * 2), ("phi_max", C.c_double),
        ("n_abs", (C.c_int64 * 5) * 2),
        ("n_cand", C.c_int64), ("n_coll", C.c_int64 * 4), ("n_see", C.c_int64),
        ("n_child", C.c_int64 * 2), ("deposit_fallback", C.c_int64),
        ("poisson", pic_poisson_stats), ("flags", C.c_int32),
        ("n_see_e", C.c_int64),
    ]

    def as_dict(self):
        d = {}
        for k, _ in self._fields_:
            v = getattr(self, k)
            if k == "n_abs":
                v = [tuple(v[s]) for s in range(2)]
            elif k == "poisson":
                v = v.as_dict()
            elif hasattr(v, "__len__"):
                v = tuple(v)
            d[k] = v
        return d


class pic_scalar_state(C.Structure):
    _fields_ = [("step", C.c_int64), ("vc", C.c_double), ("qc", C.c_double),
                ("next_id", C.c_uint32 * 2), ("count", C.c_int64 * 2),
                ("sort_phase", C.c_int32), ("ion_sort_phase", C.c_int32)]


class pic_plasma_out(C.Structure):
    _fields_ = [("z_sheath", C.c_double), ("z_bulk", C.c_double),
                ("te_region", C.c_double * 3), ("n_region", C.c_int64 * 3),
                ("lambda_d_peak", C.c_double), ("n_e_peak", C.c_double), ("te_peak", C.c_double),
                ("peak_cell", C.c_int32 * 2), ("band_cells", C.c_int32 * 2)]


class pic_timers(C.Structure):
    _fields_ = [("push_ms", C.c_double), ("children_ms", C.c_double), ("sort_ms", C.c_double),
                ("poisson_ms", C.c_double), ("circuit_ms", C.c_double), ("field_ms", C.c_double),
                ("push_launches", C.c_int64), ("sort_launches", C.c_int64),
                ("poisson_solves", C.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


EXPORTS = [
    "pic_query_workspace", "pic_init", "pic_step", "pic_poisson", "pic_diag",
    "pic_particles", "pic_fields", "pic_set_phi", "pic_compact", "pic_get_state",
    "pic_plasma_diagnostics", "pic_ied_config", "pic_ied_read", "pic_reweight",
    "pic_set_state", "pic_enable_timers", "pic_get_timers", "pic_free", "pic_last_error",
    "pic_pc_param_count", "pic_pc_set_weights", "pic_pc_get_weights", "pic_pc_train_step",
    "pic_pc_apply", "pic_set_poisson_mode", "pic_apply_operator",
    "pic_ensemble_create", "pic_ensemble_step", "pic_ensemble_free", "pic_ensemble_last_error",
    "pic_autotune", "pic_set_tuning", "pic_get_tuning", "pic_poisson_static",
]


class pic_tuning(C.Structure):
    _fields_ = [("push_blocks", C.c_int32), ("push_e_weight", C.c_double),
                ("push_ms", C.c_double), ("trials", C.c_int32),
                ("mg_one_level", C.c_int32), ("pass_graphs", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}

PIC_MGCG, PIC_LEARNED, PIC_CG, PIC_DIRECT = 0, 1, 2, 3

_lib = None


def load():
    """Load libpic.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} not found: build it with "
                           "`python -m paper_2507_10727_amd.build` (no CPU fallback exists)")
    L = C.CDLL(LIB_PATH)
    H = C.c_void_p
    L.pic_query_workspace.argtypes = [C.POINTER(pic_config), C.POINTER(C.c_int64)]
    L.pic_init.argtypes = [C.POINTER(pic_config), C.c_void_p, C.c_int64, C.c_void_p,
                           C.POINTER(pic_species_host), C.POINTER(H)]
    L.pic_step.argtypes = [H, C.c_int32]
    L.pic_poisson.argtypes = [H, C.c_void_p, C.c_double, C.c_void_p,
                              C.POINTER(pic_poisson_stats)]
    L.pic_poisson_static.argtypes = [H, C.c_void_p, C.c_double, C.c_void_p,
                                     C.POINTER(pic_poisson_stats)]
    L.pic_diag.argtypes = [H, C.POINTER(pic_diag_out)]
    L.pic_particles.argtypes = [H, C.c_int32, C.POINTER(pic_particle_view)]
    L.pic_fields.argtypes = [H, C.POINTER(pic_field_view)]
    L.pic_set_phi.argtypes = [H, _dp]
    L.pic_compact.argtypes = [H]
    L.pic_plasma_diagnostics.argtypes = [H, C.c_double, C.c_double, C.POINTER(pic_plasma_out),
                                         _dp]
    L.pic_ied_config.argtypes = [H, C.c_double, C.c_int32, C.c_double, C.c_double]
    L.pic_ied_read.argtypes = [H, C.POINTER(C.c_uint64), C.c_int32, C.c_int32]
    L.pic_reweight.argtypes = [H, C.c_int32]
    L.pic_get_state.argtypes = [H, C.POINTER(pic_scalar_state)]
    L.pic_set_state.argtypes = [H, C.POINTER(pic_scalar_state)]
    L.pic_enable_timers.argtypes = [H, C.c_int32]
    L.pic_get_timers.argtypes = [H, C.POINTER(pic_timers), C.c_int32]
    L.pic_free.argtypes = [H]
    _fp = C.POINTER(C.c_float)
    L.pic_pc_param_count.argtypes = [C.POINTER(C.c_int64)]
    L.pic_pc_set_weights.argtypes = [H, _fp, C.c_int64, C.c_double]
    L.pic_pc_get_weights.argtypes = [H, _fp, C.c_int64, C.POINTER(C.c_double)]
    L.pic_pc_train_step.argtypes = [H, C.c_void_p, C.c_void_p, C.c_int32, C.c_float,
                                    C.POINTER(C.c_double), _fp]
    L.pic_pc_apply.argtypes = [H, C.c_void_p, C.c_void_p]
    L.pic_set_poisson_mode.argtypes = [H, C.c_int32]
    L.pic_apply_operator.argtypes = [H, C.c_void_p, C.c_void_p]
    L.pic_ensemble_create.argtypes = [C.POINTER(C.c_void_p), C.c_int32, C.c_void_p, C.c_int32,
                                      C.POINTER(C.c_void_p)]
    L.pic_ensemble_step.argtypes = [C.c_void_p, C.c_int32]
    L.pic_autotune.argtypes = [H, C.c_int32, C.c_void_p, C.c_int64, C.POINTER(pic_tuning)]
    L.pic_set_tuning.argtypes = [H, C.POINTER(pic_tuning)]
    L.pic_get_tuning.argtypes = [H, C.POINTER(pic_tuning)]
    L.pic_ensemble_free.argtypes = [C.c_void_p]
    L.pic_ensemble_last_error.argtypes = [C.c_void_p]
    L.pic_ensemble_last_error.restype = C.c_char_p
    L.pic_last_error.argtypes = [H]
    L.pic_last_error.restype = C.c_char_p
    for name in EXPORTS:
        if name not in ("pic_last_error", "pic_ensemble_last_error"):
            getattr(L, name).restype = C.c_int
    _lib = L
    return L


def check(status, handle=None):
    if status != PIC_OK:
        msg = load().pic_last_error(handle)
        raise PicError(status, msg.decode() if msg else "")
    return status
