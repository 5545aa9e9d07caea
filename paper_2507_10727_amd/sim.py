"""Python front end of libpic.so.

Torch provides the device workspace and the stream; every step of the
timestep runs in the HIP library behind the C ABI.  Importing this module
never falls back to a CPU path: without the built library it raises.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib as L
from . import workloads as W


def make_config(prob: W.Problem, b_r, b_z, sigma, de_table=W.DE_TABLE, capacity=None):
    """pic_config from a Problem; returns (config, keep-alive arrays)."""
    sig = np.ascontiguousarray(sigma, np.float64)
    if sig.ndim != 2 or sig.shape[0] != 4:
        raise ValueError("sigma must hold 4 rows: elastic, excitation, ionization from the "
                         "ground state and from the metastable")
    br = np.ascontiguousarray(b_r, np.float64)
    bz = np.ascontiguousarray(b_z, np.float64)
    c = L.pic_config()
    c.nr, c.nz = prob.nr, prob.nz
    c.lr, c.lz, c.dt = prob.lr, prob.lz, prob.dt
    c.scheme, c.precision = prob.scheme, prob.precision
    c.cathode_rmax = prob.cathode_rmax
    c.circuit = prob.circuit
    c.v_fixed, c.v_ext, c.r_ext = prob.v_fixed, prob.v_ext, prob.r_ext
    c.gamma_i = prob.gamma_i
    c.gamma_e = prob.gamma_e
    c.n_meta = prob.n_meta
    c.e_iz_meta = prob.e_iz_meta
    c.deposit_fixed = prob.deposit_fixed
    c.pc_pre = prob.pc_pre
    c.p_gas, c.t_gas = prob.p_gas, prob.t_gas
    c.e_exc, c.e_iz = prob.e_exc, prob.e_iz
    c.sigma = sig.ctypes.data_as(C.POINTER(C.c_double))
    c.n_table = sig.shape[1]
    c.de_table = de_table
    c.b_r = br.ctypes.data_as(C.POINTER(C.c_double))
    c.b_z = bz.ctypes.data_as(C.POINTER(C.c_double))
    for s, (q, m, w) in enumerate(prob.species()):
        c.q[s], c.m[s], c.w[s] = q, m, w
    c.seed = prob.seed
    c.run = prob.run
    cap = capacity or prob.capacity()
    c.capacity[0], c.capacity[1] = int(cap[0]), int(cap[1])
    c.sort_every = prob.sort_every
    c.poisson_mode = prob.poisson_mode
    c.pc_batch = prob.pc_batch
    c.pc_maxit = prob.pc_maxit
    c.poisson_rtol = prob.poisson_rtol
    c.poisson_maxit = prob.poisson_maxit
    for k in range(3):
        c.wall_bc[k] = prob.wall_bc[k]
    c.frozen_ions, c.mcc_on, c.see_on = prob.frozen_ions, prob.mcc_on, prob.see_on
    c.field_solve = prob.field_solve
    c.extra_current = prob.extra_current
    return c, (sig, br, bz)


def workspace_bytes(prob: W.Problem, b_r, b_z, sigma, capacity=None) -> int:
    """Device bytes a Simulation of prob needs (pic_query_workspace)."""
    cfg, keep = make_config(prob, b_r, b_z, sigma, capacity=capacity)
    nbytes = C.c_int64()
    L.check(L.load().pic_query_workspace(C.byref(cfg), C.byref(nbytes)))
    del keep
    return int(nbytes.value)


def unpack_positions(h, pos_bits):
    """key (j << 16 | i, -1 absorbed), fr, fz from host copies of a species'
    arrays: as stored (FP64 state) or decoded from the packed FP32 words."""
    if not pos_bits:
        return {"key": h["key"], "fr": h["fr"], "fz": h["fz"]}
    pr = h["pr"].view(np.uint32).astype(np.int64)
    pz = h["pz"].astype(np.int64)
    mask = (1 << pos_bits) - 1
    scale = np.float32(1.0 / (1 << pos_bits))
    live = pz >= 0
    i = pr >> pos_bits
    j = np.where(live, pz, 0) >> pos_bits
    key = np.where(live, (j << 16) | i, -1).astype(np.int32)
    fr = (pr & mask).astype(np.float32) * scale
    fz = np.where(live, (np.where(live, pz, 0) & mask).astype(np.float32) * scale, np.float32(0))
    return {"key": key, "fr": fr, "fz": fz.astype(np.float32)}


class Simulation:
    """One discharge on one GPU.

    ``particles`` is a pair of :class:`workloads.SpeciesArrays` (host FP64,
    absolute positions) or None.
    """

    def __init__(self, prob: W.Problem, b_r, b_z, sigma, particles=None, device="cuda:0",
                 capacity=None, timers=False, workspace=None):
        import torch

        self.torch = torch
        self.prob = prob
        self.lib = L.load()
        self.device = torch.device(device)
        cfg, keep = make_config(prob, b_r, b_z, sigma, capacity=capacity)
        self.cfg = cfg
        nbytes = C.c_int64()
        L.check(self.lib.pic_query_workspace(C.byref(cfg), C.byref(nbytes)))
        if workspace is None:
            self.ws = torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.device)
        else:
            # caller-provided device bytes (e.g. a slice of a larger buffer)
            if (workspace.dtype != torch.uint8 or not workspace.is_cuda
                    or workspace.numel() < nbytes.value or workspace.data_ptr() % 256):
                raise ValueError(f"workspace must be a 256-byte aligned CUDA uint8 tensor of at "
                                 f"least {nbytes.value} bytes")
            self.ws = workspace
        # a stream of our own (default priority): the library captures its
        # field-solve passes as graphs, which the legacy null stream forbids
        self.stream = torch.cuda.Stream(device=self.device)
        torch.cuda.synchronize(self.device)
        hosts = (L.pic_species_host * 2)()
        keep_p = []
        if particles is not None:
            for s in range(2):
                p = particles[s]
                arrs = [np.ascontiguousarray(getattr(p, k), np.float64)
                        for k in ("r", "z", "vr", "vt", "vz")]
                ids = np.ascontiguousarray(p.id, np.uint32)
                keep_p.append((arrs, ids))
                h = hosts[s]
                h.r, h.z, h.vr, h.vt, h.vz = (a.ctypes.data_as(C.POINTER(C.c_double)) for a in arrs)
                h.id = ids.ctypes.data_as(C.POINTER(C.c_uint32))
                h.n = p.n
        handle = C.c_void_p()
        status = self.lib.pic_init(C.byref(cfg), C.c_void_p(self.ws.data_ptr()), nbytes.value,
                                   C.c_void_p(self.stream.cuda_stream),
                                   hosts if particles is not None else None, C.byref(handle))
        L.check(status, None)
        self.h = handle
        del keep, keep_p
        if timers:
            L.check(self.lib.pic_enable_timers(self.h, 1), self.h)

    # -- stepping ------------------------------------------------------------
    def step(self, n=1):
        L.check(self.lib.pic_step(self.h, int(n)), self.h)

    def diag(self):
        d = L.pic_diag_out()
        L.check(self.lib.pic_diag(self.h, C.byref(d)), self.h)
        return d.as_dict()

    def compact(self):
        L.check(self.lib.pic_compact(self.h), self.h)

    def poisson(self, q, v_cathode, phi):
        """Solve K phi = q in place on device tensors (float64); returns stats."""
        self.torch.cuda.synchronize(self.device)
        st = L.pic_poisson_stats()
        status = self.lib.pic_poisson(self.h, C.c_void_p(q.data_ptr()), float(v_cathode),
                                      C.c_void_p(phi.data_ptr()), C.byref(st))
        L.check(status, self.h)
        return st.as_dict()

    def poisson_static(self, q, v_cathode, phi):
        """pic_poisson_static: the direct solve with the library's static
        scratch (allocates nothing); returns (status, stats)."""
        self.torch.cuda.synchronize(self.device)
        st = L.pic_poisson_stats()
        status = self.lib.pic_poisson_static(self.h, C.c_void_p(q.data_ptr()), float(v_cathode),
                                             C.c_void_p(phi.data_ptr()), C.byref(st))
        return status, st.as_dict()

    def poisson_status(self, q, v_cathode, phi):
        self.torch.cuda.synchronize(self.device)
        st = L.pic_poisson_stats()
        status = self.lib.pic_poisson(self.h, C.c_void_p(q.data_ptr()), float(v_cathode),
                                      C.c_void_p(phi.data_ptr()), C.byref(st))
        return status, st.as_dict()

    def set_phi(self, phi):
        a = np.ascontiguousarray(phi, np.float64)
        L.check(self.lib.pic_set_phi(self.h, a.ctypes.data_as(C.POINTER(C.c_double))), self.h)

    def get_state(self):
        s = L.pic_scalar_state()
        L.check(self.lib.pic_get_state(self.h, C.byref(s)), self.h)
        return {"step": s.step, "vc": s.vc, "qc": s.qc, "next_id": tuple(s.next_id),
                "count": tuple(s.count), "sort_phase": s.sort_phase,
                "ion_sort_phase": s.ion_sort_phase}

    def set_state(self, st):
        s = L.pic_scalar_state()
        s.step, s.vc, s.qc = st["step"], st["vc"], st["qc"]
        s.next_id[0], s.next_id[1] = st["next_id"]
        s.count[0], s.count[1] = st["count"]
        s.sort_phase = st.get("sort_phase", 0)
        s.ion_sort_phase = st.get("ion_sort_phase", 0)
        L.check(self.lib.pic_set_state(self.h, C.byref(s)), self.h)

    # -- plasma diagnostics ---------------------------------------------------
    def plasma_diagnostics(self, r0, r1, maps=False):
        """Region temperatures, sheath and bulk edges over the band of cells
        with centres in [r0, r1), the Debye length at the density peak and,
        with maps=True, the cell maps (n_e, n_i, T_e, lambda_D; each nz x nr)."""
        o = L.pic_plasma_out()
        buf = np.zeros(4 * self.prob.nr * self.prob.nz) if maps else None
        ptr = buf.ctypes.data_as(C.POINTER(C.c_double)) if maps else None
        L.check(self.lib.pic_plasma_diagnostics(self.h, float(r0), float(r1), C.byref(o), ptr),
                self.h)
        out = {"z_sheath": o.z_sheath, "z_bulk": o.z_bulk, "te_region": list(o.te_region),
               "n_region": list(o.n_region), "lambda_d_peak": o.lambda_d_peak,
               "n_e_peak": o.n_e_peak, "te_peak": o.te_peak,
               "peak_cell": tuple(o.peak_cell), "band_cells": tuple(o.band_cells)}
        if maps:
            m = buf.reshape(4, self.prob.nz, self.prob.nr)
            out["maps"] = {"n_e": m[0], "n_i": m[1], "te": m[2], "lambda_d": m[3]}
        return out

    def ied_config(self, emax_ev, nbins, r0, r1):
        L.check(self.lib.pic_ied_config(self.h, float(emax_ev), int(nbins), float(r0),
                                        float(r1)), self.h)
        self._ied_bins = int(nbins)

    def ied(self, reset=False):
        a = np.zeros(self._ied_bins + 1, np.uint64)
        L.check(self.lib.pic_ied_read(self.h, a.ctypes.data_as(C.POINTER(C.c_uint64)),
                                      a.shape[0], int(bool(reset))), self.h)
        return a

    def reweight(self, keep_every):
        L.check(self.lib.pic_reweight(self.h, int(keep_every)), self.h)

    def checkpoint(self):
        """Host copy of everything a resumed run needs: the scalar state, the
        used slots of both species' arrays, phi0 and phi0_prev."""
        st = self.get_state()
        ck = {"state": st}
        for s in range(2):
            t = self.particle_tensors(s)
            ck[f"species{s}"] = {k: v.cpu().clone() for k, v in t.items()}
        f = self.fields()
        ck["phi0"] = f["phi0"].cpu().clone()
        ck["phi0_prev"] = f["phi0_prev"].cpu().clone()
        return ck

    def restore(self, ck):
        """Write a checkpoint into this simulation (same configuration): the
        arrays through the views, then the scalar state, which rebuilds phi
        and the gather fields."""
        torch = self.torch
        for s in range(2):
            src = ck[f"species{s}"]
            n = int(ck["state"]["count"][s])
            v = L.pic_particle_view()
            L.check(self.lib.pic_particles(self.h, int(s), C.byref(v)), self.h)
            if n > v.capacity:
                raise ValueError(f"species {s}: {n} particles exceed capacity {v.capacity}")
            ft = torch.float64 if v.precision == 1 else torch.float32
            dst = {"id": self._view(v.id_dev, n, torch.int32)}
            if v.pos_bits:
                dst["pr"] = self._view(v.fr_dev, n, torch.int32)
                dst["pz"] = self._view(v.fz_dev, n, torch.int32)
            else:
                dst["key"] = self._view(v.key_dev, n, torch.int32)
                dst["fr"] = self._view(v.fr_dev, n, ft)
                dst["fz"] = self._view(v.fz_dev, n, ft)
            for k in ("vr", "vt", "vz"):
                dst[k] = self._view(getattr(v, k + "_dev"), n, ft)
            if dst.keys() != src.keys():
                raise ValueError("checkpoint taken with another state precision")
            for k in dst:
                dst[k].copy_(src[k][:n].to(self.device))
        f = self.fields()
        f["phi0"].copy_(ck["phi0"].to(self.device))
        f["phi0_prev"].copy_(ck["phi0_prev"].to(self.device))
        torch.cuda.synchronize(self.device)
        self.set_state(ck["state"])

    # -- learned preconditioner ----------------------------------------------
    def pc_param_count(self):
        n = C.c_int64()
        L.check(self.lib.pic_pc_param_count(C.byref(n)), self.h)
        return int(n.value)

    def pc_set_weights(self, theta, out_scale):
        a = np.ascontiguousarray(theta, np.float32)
        L.check(self.lib.pic_pc_set_weights(self.h, a.ctypes.data_as(C.POINTER(C.c_float)),
                                            a.size, float(out_scale)), self.h)

    def pc_get_weights(self):
        a = np.zeros(self.pc_param_count(), np.float32)
        sc = C.c_double()
        L.check(self.lib.pic_pc_get_weights(self.h, a.ctypes.data_as(C.POINTER(C.c_float)),
                                            a.size, C.byref(sc)), self.h)
        return a, sc.value

    def pc_train_step(self, q, phi, lr, want_grad=False):
        """One Adam step on device tensors q, phi (float64, [batch, nodes]);
        returns the loss before the update (and the gradient if asked)."""
        self.torch.cuda.synchronize(self.device)
        loss = C.c_double()
        g = np.zeros(self.pc_param_count(), np.float32) if want_grad else None
        gp = g.ctypes.data_as(C.POINTER(C.c_float)) if want_grad else None
        L.check(self.lib.pic_pc_train_step(self.h, C.c_void_p(q.data_ptr()),
                                           C.c_void_p(phi.data_ptr()), int(q.shape[0]),
                                           float(lr), C.byref(loss), gp), self.h)
        return (loss.value, g) if want_grad else loss.value

    def pc_apply(self, r, z):
        self.torch.cuda.synchronize(self.device)
        L.check(self.lib.pic_pc_apply(self.h, C.c_void_p(r.data_ptr()), C.c_void_p(z.data_ptr())),
                self.h)

    def apply_operator(self, phi, out):
        """out = K phi (device float64 tensors)."""
        self.torch.cuda.synchronize(self.device)
        L.check(self.lib.pic_apply_operator(self.h, C.c_void_p(phi.data_ptr()),
                                            C.c_void_p(out.data_ptr())), self.h)

    def autotune(self, steps_per_trial=2, restore=True):
        """Time launch shapes on the live run (pic_autotune); with restore,
        the run's state is copied to a scratch tensor of the workspace's
        size first and put back afterwards."""
        t = L.pic_tuning()
        scratch, nbytes = None, 0
        if restore:
            scratch = self.torch.empty_like(self.ws)
            nbytes = scratch.numel()
        L.check(self.lib.pic_autotune(self.h, int(steps_per_trial),
                                      C.c_void_p(scratch.data_ptr() if scratch is not None else None),
                                      C.c_int64(nbytes), C.byref(t)), self.h)
        del scratch
        return t.as_dict()

    def set_tuning(self, push_blocks=None, push_e_weight=None, mg_one_level=None,
                   pass_graphs=None):
        """Apply launch choices; a field left None keeps its current value."""
        t = L.pic_tuning()
        L.check(self.lib.pic_get_tuning(self.h, C.byref(t)), self.h)
        if pass_graphs is not None:
            t.pass_graphs = int(pass_graphs)
        if push_blocks is not None:
            t.push_blocks = int(push_blocks)
        if push_e_weight is not None:
            t.push_e_weight = float(push_e_weight)
        if mg_one_level is not None:
            t.mg_one_level = int(mg_one_level)
        L.check(self.lib.pic_set_tuning(self.h, C.byref(t)), self.h)

    def tuning(self):
        t = L.pic_tuning()
        L.check(self.lib.pic_get_tuning(self.h, C.byref(t)), self.h)
        return t.as_dict()

    def set_poisson_mode(self, mode):
        L.check(self.lib.pic_set_poisson_mode(self.h, int(mode)), self.h)

    def timers(self, reset=True):
        t = L.pic_timers()
        L.check(self.lib.pic_get_timers(self.h, C.byref(t), int(reset)), self.h)
        return t.as_dict()

    # -- views into the workspace -------------------------------------------
    def _view(self, ptr, n, dtype):
        torch = self.torch
        esz = torch.empty(0, dtype=dtype).element_size()
        off = int(ptr) - self.ws.data_ptr()
        assert 0 <= off and off + n * esz <= self.ws.numel()
        return self.ws[off:off + n * esz].view(dtype)

    def particle_tensors(self, s):
        """Device views of species s's arrays (slots 0..count-1).  FP64
        state: key, fr, fz, ...; FP32 state: the packed words pr, pz (see
        pic_particle_view) instead of key, fr, fz."""
        v = L.pic_particle_view()
        L.check(self.lib.pic_particles(self.h, int(s), C.byref(v)), self.h)
        torch = self.torch
        ft = torch.float64 if v.precision == 1 else torch.float32
        n = int(v.count)
        out = {"id": self._view(v.id_dev, n, torch.int32)}
        if v.pos_bits:
            out["pr"] = self._view(v.fr_dev, n, torch.int32)
            out["pz"] = self._view(v.fz_dev, n, torch.int32)
        else:
            out["key"] = self._view(v.key_dev, n, torch.int32)
            out["fr"] = self._view(v.fr_dev, n, ft)
            out["fz"] = self._view(v.fz_dev, n, ft)
        for k in ("vr", "vt", "vz"):
            out[k] = self._view(getattr(v, k + "_dev"), n, ft)
        self._pos_bits = int(v.pos_bits)
        return out

    def particles(self, s, raw=False):
        """Live particles of species s as host arrays (positions absolute, FP64)."""
        t = self.particle_tensors(s)
        self.torch.cuda.synchronize(self.device)
        h = {k: v.cpu().numpy() for k, v in t.items()}
        h.update(unpack_positions(h, self._pos_bits))
        live = h["key"] >= 0
        out = {k: h[k][live] for k in ("key", "fr", "fz", "vr", "vt", "vz", "id")}
        out["id"] = out["id"].view(np.uint32)
        i = (out["key"] & 0xFFFF).astype(np.float64)
        j = (out["key"] >> 16).astype(np.float64)
        out["i"] = i.astype(np.int64)
        out["j"] = j.astype(np.int64)
        out["r"] = (i + out["fr"].astype(np.float64)) * self.prob.dr
        out["z"] = (j + out["fz"].astype(np.float64)) * self.prob.dz
        for k in ("vr", "vt", "vz", "fr", "fz"):
            out[k] = out[k].astype(np.float64)
        return out

    def fields(self):
        v = L.pic_field_view()
        L.check(self.lib.pic_fields(self.h, C.byref(v)), self.h)
        torch = self.torch
        n = int(v.nodes)
        qt = torch.float64 if v.q_precision == 1 else torch.float32
        return {"phi": self._view(v.phi_dev, n, torch.float64),
                "phi0": self._view(v.phi0_dev, n, torch.float64),
                "phi0_prev": self._view(v.phi0_prev_dev, n, torch.float64),
                "phi_l": self._view(v.phi_l_dev, n, torch.float64),
                "q_e": self._view(v.q_dev[0], n, qt), "q_i": self._view(v.q_dev[1], n, qt)}

    def fields_host(self):
        self.torch.cuda.synchronize(self.device)
        return {k: v.cpu().numpy().astype(np.float64) for k, v in self.fields().items()}

    def close(self):
        if getattr(self, "h", None):
            self.lib.pic_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Ensemble:
    """Independent Simulations advanced together: one step of all of them is
    a single replay of a captured hipGraph (see pic_ensemble_create)."""

    def __init__(self, sims, nstreams=4):
        import torch

        self.torch = torch
        self.sims = list(sims)
        self.lib = L.load()
        arr = (C.c_void_p * len(self.sims))(*[s.h.value for s in self.sims])
        self.stream = torch.cuda.Stream(device=self.sims[0].device)
        e = C.c_void_p()
        st = self.lib.pic_ensemble_create(arr, len(self.sims), C.c_void_p(self.stream.cuda_stream),
                                          int(nstreams), C.byref(e))
        self._check(st, None)
        self.e = e

    def _check(self, status, e):
        if status != L.PIC_OK:
            msg = self.lib.pic_ensemble_last_error(e)
            raise L.PicError(status, msg.decode() if msg else "")

    def step(self, n=1):
        self._check(self.lib.pic_ensemble_step(self.e, int(n)), self.e)

    def close(self):
        if getattr(self, "e", None):
            self.lib.pic_ensemble_free(self.e)
            self.e = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
