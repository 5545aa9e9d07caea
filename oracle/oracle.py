"""ctypes wrapper around the FP64 CPU oracle (TEST INFRASTRUCTURE ONLY).

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's
``cpu_baseline`` leg may import this module.  The GPU library never does.

``build()`` compiles ``pic_oracle.c`` with gcc (``-O2 -ffp-contract=off
-fno-fast-math``) into ``liborc.so`` next to this file.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "pic_oracle.c")
LIB = os.path.join(HERE, "liborc.so")
LIB_OMP = os.path.join(HERE, "liborc_omp.so")

_dp = C.POINTER(C.c_double)
_up = C.POINTER(C.c_uint32)
_up64 = C.POINTER(C.c_uint64)


class Problem(C.Structure):
    _fields_ = [
        ("nr", C.c_int32), ("nz", C.c_int32),
        ("lr", C.c_double), ("lz", C.c_double), ("dt", C.c_double),
        ("scheme", C.c_int32),
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
        ("wall_bc", C.c_int32 * 3),
        ("frozen_ions", C.c_int32), ("mcc_on", C.c_int32), ("see_on", C.c_int32),
        ("field_solve", C.c_int32),
        ("extra_current", C.c_double),
        ("poisson_rtol", C.c_double), ("poisson_maxit", C.c_int32),
        ("gamma_e", C.c_double), ("n_meta", C.c_double), ("e_iz_meta", C.c_double),
        ("ied_emax", C.c_double), ("ied_r0", C.c_double), ("ied_r1", C.c_double),
        ("ied_nbins", C.c_int32), ("ied_hist", _up64),
    ]


class Species(C.Structure):
    _fields_ = [("r", _dp), ("z", _dp), ("vr", _dp), ("vt", _dp), ("vz", _dp),
                ("id", _up), ("n", C.c_int64), ("cap", C.c_int64)]


class State(C.Structure):
    _fields_ = [("step", C.c_int64), ("vc", C.c_double), ("qc", C.c_double),
                ("cap_c", C.c_double), ("next_id", C.c_uint32 * 2)]


class Diag(C.Structure):
    _fields_ = [("ke", C.c_double * 2), ("pz", C.c_double * 2), ("w_field", C.c_double),
                ("q_dep", C.c_double * 2), ("dq_conv", C.c_double), ("qc0", C.c_double),
                ("n_abs", (C.c_int64 * 5) * 2), ("n_cand", C.c_int64),
                ("n_coll", C.c_int64 * 4), ("n_see", C.c_int64),
                ("n_child", C.c_int64 * 2), ("poisson_iters", C.c_int64),
                ("poisson_res", C.c_double), ("n_peak", C.c_double * 2),
                ("phi_max", C.c_double), ("i_cathode", C.c_double),
                ("n_see_e", C.c_int64)]

    def as_dict(self):
        return {
            "ke": tuple(self.ke), "pz": tuple(self.pz), "w_field": self.w_field,
            "q_dep": tuple(self.q_dep), "dq_conv": self.dq_conv, "qc0": self.qc0,
            "n_abs": [tuple(self.n_abs[s]) for s in range(2)],
            "n_cand": self.n_cand, "n_coll": tuple(self.n_coll), "n_see": self.n_see,
            "n_child": tuple(self.n_child), "poisson_iters": self.poisson_iters,
            "poisson_res": self.poisson_res, "n_peak": tuple(self.n_peak),
            "phi_max": self.phi_max, "i_cathode": self.i_cathode, "n_see_e": self.n_see_e,
        }


_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (always rebuilds when ``force``): the serial
    library liborc.so, and liborc_omp.so with OpenMP over the particle loops
    (the multi-core timing build)."""
    for out, extra in ((LIB, []), (LIB_OMP, ["-fopenmp"])):
        if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(SRC):
            tmp = out + ".tmp"
            subprocess.check_call([
                "gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11",
                "-fPIC", "-shared", *extra, "-o", tmp, SRC, "-lm"])
            os.replace(tmp, out)
    return LIB


def use_openmp(on: bool = True):
    """Select the OpenMP build for the oracle runs that follow (timing only;
    the parity tests use the serial build).  Oracle objects made before the
    switch must not be used after it."""
    global _which, _lib
    want = LIB_OMP if on else LIB
    if (_which or LIB) != want:
        _lib = None
    _which = want


def thread_count() -> int:
    """Threads the loaded build runs its particle loops on."""
    return int(lib().orc_thread_count())


_which = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(_which or LIB)
        L.orc_philox4x32_10.argtypes = [_up, _up, _up]
        L.orc_node_kind.argtypes = [C.POINTER(Problem), C.c_int, C.c_int]
        L.orc_node_kind.restype = C.c_int
        L.orc_couplings.argtypes = [C.POINTER(Problem), _dp, _dp]
        L.orc_apply_k_full.argtypes = [C.POINTER(Problem), _dp, _dp]
        L.orc_solve.argtypes = [C.POINTER(Problem), _dp, C.c_double, _dp, C.c_double,
                                C.c_int, C.POINTER(C.c_int64), C.POINTER(C.c_double)]
        L.orc_solve.restype = C.c_int
        L.orc_field_energy.argtypes = [C.POINTER(Problem), _dp]
        L.orc_field_energy.restype = C.c_double
        L.orc_nodal_e.argtypes = [C.POINTER(Problem), _dp, _dp, _dp]
        L.orc_deposit.argtypes = [C.POINTER(Problem), _dp, _dp, C.c_int64, C.c_double, _dp]
        L.orc_gather.argtypes = [C.POINTER(Problem), _dp, _dp, _dp, C.c_int64, _dp, _dp, _dp, _dp]
        L.orc_nu_tables.argtypes = [C.POINTER(Problem), _dp, C.POINTER(C.c_uint64)]
        L.orc_nu_tables.restype = C.c_double
        L.orc_node_volumes.argtypes = [C.POINTER(Problem), _dp]
        L.orc_capacitance.argtypes = [C.POINTER(Problem), _dp]
        L.orc_capacitance.restype = C.c_double
        L.orc_induced_charge.argtypes = [C.POINTER(Problem), _dp, _dp]
        L.orc_induced_charge.restype = C.c_double
        L.orc_mcc_select.argtypes = [C.POINTER(Problem), _dp, C.c_double, C.c_uint64, C.c_uint32,
                                     C.c_int64, C.c_double, C.c_double, C.c_double,
                                     C.POINTER(C.c_double)]
        L.orc_mcc_select.restype = C.c_int
        L.orc_mcc_select_many.argtypes = [C.POINTER(Problem), C.c_int64, C.c_int64, _up, _dp, _dp,
                                          _dp, C.POINTER(C.c_int32), _dp]
        L.orc_init.argtypes = [C.POINTER(Problem), C.POINTER(Species), C.POINTER(State),
                               _dp, _dp, _dp, _dp, _dp]
        L.orc_init.restype = C.c_int
        L.orc_step.argtypes = [C.POINTER(Problem), C.POINTER(Species), C.POINTER(State),
                               _dp, _dp, _dp, _dp, _dp, C.POINTER(Diag)]
        L.orc_step.restype = C.c_int
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(_dp)


def _u(a):
    return a.ctypes.data_as(_up)


def philox(ctr, key):
    """Philox4x32-10 of one 4-word counter and 2-word key -> 4 uint32."""
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    o = np.zeros(4, np.uint32)
    lib().orc_philox4x32_10(_u(c), _u(k), _u(o))
    return o


class Oracle:
    """An oracle run: a problem, two species with capacity, grids and state.

    ``prob`` is a :class:`paper_2507_10727_amd.workloads.Problem`; the static
    field, cross sections and particles are passed in (the oracle generates
    nothing itself).
    """

    def __init__(self, prob, b_r, b_z, sigma, particles=None, capacity=None, rtol=None):
        self.prob = prob
        self.b_r = np.ascontiguousarray(b_r, np.float64)
        self.b_z = np.ascontiguousarray(b_z, np.float64)
        self.sigma = np.ascontiguousarray(sigma, np.float64)
        P = Problem()
        P.nr, P.nz = prob.nr, prob.nz
        P.lr, P.lz, P.dt = prob.lr, prob.lz, prob.dt
        P.scheme = prob.scheme
        P.cathode_rmax = prob.cathode_rmax
        P.circuit = prob.circuit
        P.v_fixed, P.v_ext, P.r_ext = prob.v_fixed, prob.v_ext, prob.r_ext
        P.gamma_i = prob.gamma_i
        P.gamma_e = prob.gamma_e
        P.n_meta = prob.n_meta
        P.e_iz_meta = prob.e_iz_meta
        P.p_gas, P.t_gas = prob.p_gas, prob.t_gas
        P.e_exc, P.e_iz = prob.e_exc, prob.e_iz
        P.sigma = _d(self.sigma)
        P.n_table = self.sigma.shape[1]
        P.de_table = 0.05 if not hasattr(prob, "de_table") else prob.de_table
        P.b_r, P.b_z = _d(self.b_r), _d(self.b_z)
        sp = prob.species()
        for s in range(2):
            P.q[s], P.m[s], P.w[s] = sp[s]
        P.seed = prob.seed
        P.run = prob.run
        for k in range(3):
            P.wall_bc[k] = prob.wall_bc[k]
        P.frozen_ions, P.mcc_on, P.see_on = prob.frozen_ions, prob.mcc_on, prob.see_on
        P.field_solve = prob.field_solve
        P.extra_current = prob.extra_current
        # FP64 conjugate gradients reach ~1e-13 relative residual on the small
        # grids; on large grids round-off in phi limits smooth problems to
        # roughly eps * condition number, so a looser target is used there.
        if rtol is None:
            rtol = 1e-13 if prob.nodes <= 20000 else 1e-10
        P.poisson_rtol = rtol
        P.poisson_maxit = 200000
        self.P = P
        nn = prob.nodes
        self.phi = np.zeros(nn)
        self.phi0 = np.zeros(nn)
        self.phi_l = np.zeros(nn)
        self.q = [np.zeros(nn), np.zeros(nn)]
        self.state = State()
        cap = capacity or prob.capacity()
        self.arrays = []
        self.S = (Species * 2)()
        for s in range(2):
            c = int(cap[s])
            arrs = {k: np.zeros(c) for k in ("r", "z", "vr", "vt", "vz")}
            arrs["id"] = np.zeros(c, np.uint32)
            n = 0
            if particles is not None:
                src = particles[s]
                n = src.n
                if n > c:
                    raise ValueError("capacity too small")
                for k in ("r", "z", "vr", "vt", "vz", "id"):
                    arrs[k][:n] = getattr(src, k)
            self.arrays.append(arrs)
            S = self.S[s]
            S.r, S.z, S.vr, S.vt, S.vz = (_d(arrs[k]) for k in ("r", "z", "vr", "vt", "vz"))
            S.id = _u(arrs["id"])
            S.n, S.cap = n, c

    def ied_config(self, emax_ev, nbins, r0, r1):
        """Record the energies of Ar+ absorbed by the cathode with r0 <= r <
        r1 (Section 7) in nbins bins over [0, emax_ev) plus an overflow bin,
        from the next step on."""
        self.ied_hist = np.zeros(int(nbins) + 1, np.uint64)
        self.P.ied_emax, self.P.ied_r0, self.P.ied_r1 = emax_ev, r0, r1
        self.P.ied_nbins = int(nbins)
        self.P.ied_hist = self.ied_hist.ctypes.data_as(_up64)

    def ied(self):
        return self.ied_hist.copy()

    def reweight(self, k):
        """Keep the particles whose id is a multiple of k and multiply both
        species' weight by k (one in k kept, expected charge unchanged)."""
        from oracle import diagnostics as D
        for s in range(2):
            n = self.S[s].n
            a = self.arrays[s]
            keep = D.reweight_keep(a["id"][:n], k)
            m = int(keep.sum())
            for key in a:
                a[key][:m] = a[key][:n][keep]
            self.S[s].n = m
            self.P.w[s] *= k

    def init(self):
        rc = lib().orc_init(C.byref(self.P), self.S, C.byref(self.state), _d(self.phi),
                            _d(self.phi0), _d(self.phi_l), _d(self.q[0]), _d(self.q[1]))
        return rc

    def step(self):
        d = Diag()
        rc = lib().orc_step(C.byref(self.P), self.S, C.byref(self.state), _d(self.phi),
                            _d(self.phi0), _d(self.phi_l), _d(self.q[0]), _d(self.q[1]),
                            C.byref(d))
        if rc not in (0,):
            raise RuntimeError(f"oracle step failed rc={rc}")
        return d.as_dict()

    def count(self, s):
        return int(self.S[s].n)

    def particles(self, s):
        n = self.count(s)
        return {k: v[:n].copy() for k, v in self.arrays[s].items()}

    def set_state(self, step=None, vc=None):
        if step is not None:
            self.state.step = step
        if vc is not None:
            self.state.vc = vc

    # -- pieces --------------------------------------------------------------
    def couplings(self):
        ce = np.zeros(self.prob.nodes)
        cn = np.zeros(self.prob.nodes)
        lib().orc_couplings(C.byref(self.P), _d(ce), _d(cn))
        return ce, cn

    def node_kind(self):
        p = self.prob
        k = np.zeros((p.nz + 1, p.nr + 1), np.int32)
        for j in range(p.nz + 1):
            for i in range(p.nr + 1):
                k[j, i] = lib().orc_node_kind(C.byref(self.P), i, j)
        return k.ravel()

    def apply_k(self, phi):
        phi = np.ascontiguousarray(phi, np.float64)
        out = np.zeros_like(phi)
        lib().orc_apply_k_full(C.byref(self.P), _d(phi), _d(out))
        return out

    def solve(self, q_node, v_cathode=0.0, phi0=None, rtol=1e-13, maxit=200000):
        q_node = np.ascontiguousarray(q_node, np.float64)
        phi = np.zeros(self.prob.nodes) if phi0 is None else np.array(phi0, np.float64)
        it = C.c_int64()
        res = C.c_double()
        rc = lib().orc_solve(C.byref(self.P), _d(q_node), v_cathode, _d(phi), rtol, maxit,
                             C.byref(it), C.byref(res))
        return phi, rc, it.value, res.value

    def field_energy(self, phi):
        phi = np.ascontiguousarray(phi, np.float64)
        return lib().orc_field_energy(C.byref(self.P), _d(phi))

    def nodal_e(self, phi):
        phi = np.ascontiguousarray(phi, np.float64)
        er = np.zeros_like(phi)
        ez = np.zeros_like(phi)
        lib().orc_nodal_e(C.byref(self.P), _d(phi), _d(er), _d(ez))
        return er, ez

    def deposit(self, r, z, qw):
        r = np.ascontiguousarray(r, np.float64)
        z = np.ascontiguousarray(z, np.float64)
        out = np.zeros(self.prob.nodes)
        lib().orc_deposit(C.byref(self.P), _d(r), _d(z), r.shape[0], qw, _d(out))
        return out

    def gather(self, phi, r, z):
        phi = np.ascontiguousarray(phi, np.float64)
        r = np.ascontiguousarray(r, np.float64)
        z = np.ascontiguousarray(z, np.float64)
        n = r.shape[0]
        out = [np.zeros(n) for _ in range(4)]
        lib().orc_gather(C.byref(self.P), _d(phi), _d(r), _d(z), n, *(_d(o) for o in out))
        return out

    def node_volumes(self):
        v = np.zeros(self.prob.nodes)
        lib().orc_node_volumes(C.byref(self.P), _d(v))
        return v

    def capacitance(self, phi_l):
        phi_l = np.ascontiguousarray(phi_l, np.float64)
        return lib().orc_capacitance(C.byref(self.P), _d(phi_l))

    def induced_charge(self, phi0, q_node):
        phi0 = np.ascontiguousarray(phi0, np.float64)
        q_node = np.ascontiguousarray(q_node, np.float64)
        return lib().orc_induced_charge(C.byref(self.P), _d(phi0), _d(q_node))

    def mcc_select(self, ids, step, vr, vt, vz):
        """The oracle's null-collision decision for each electron (ids, velocities
        after the push): codes -2 not a candidate, -1 null, 0/1/2 process, and the
        relative margin of the deciding floating-point comparisons."""
        ids = np.ascontiguousarray(ids, np.uint32)
        vr, vt, vz = (np.ascontiguousarray(a, np.float64) for a in (vr, vt, vz))
        n = ids.shape[0]
        code = np.zeros(n, np.int32)
        margin = np.zeros(n)
        lib().orc_mcc_select_many(C.byref(self.P), int(step), n, _u(ids), _d(vr), _d(vt), _d(vz),
                                  code.ctypes.data_as(C.POINTER(C.c_int32)), _d(margin))
        return code, margin

    def nu_tables(self):
        nu = np.zeros((4, self.sigma.shape[1]))
        t = C.c_uint64()
        numax = lib().orc_nu_tables(C.byref(self.P), _d(nu), C.byref(t))
        return nu, numax, t.value
