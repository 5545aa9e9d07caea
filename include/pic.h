/*
 * pic.h -- C ABI of libpic.so: one explicit electrostatic 2D R-Z PIC-MCC
 * timestep of a dc magnetron discharge on an AMD Instinct MI355X (gfx950).
 *
 * The method is the one of Main et al., "Modeling the Role of Secondary
 * Electron Emission in Direct Current Magnetron Sputtering using Explicit
 * Energy-Conserving Particle-in-Cell Methods" (arXiv 2507.10727):
 *   Section 2 -- momentum-conserving (MC-PIC) and energy-conserving (EC-PIC)
 *                field gathers; nodal potential and charge, edge-centred E;
 *                linear (tent) charge deposition;
 *   Section 3 -- R-Z geometry with azimuthal symmetry; grounded anode at
 *                z = Z_max; cathode on z = 0 floating through an external
 *                circuit, with a Neumann block beside it; Gauss's law on the
 *                axis; absorbing z and outer-r walls, reflective axis;
 *                constant ion-induced secondary electron yield with electrons
 *                emitted at rest; Monte Carlo collisions of electrons with a
 *                static argon background (elastic, excitation, ground-state
 *                ionization);
 *   Section 4 -- uniform seed load; external resistor circuit.
 *
 * Conventions
 *   - All units SI; energies of the collision tables in eV.
 *   - Grid sizes count CELLS: nodes are (nr+1) x (nz+1); node (i, j) sits at
 *     r = i*dr, z = j*dz and is stored at linear index j*(nr+1) + i.
 *   - Species 0 = electrons, 1 = Ar+.
 *   - Pointers named *_dev are device pointers (hipMalloc'd or torch CUDA
 *     tensors); every other pointer is host memory.
 *   - The library never allocates device memory: the caller passes one
 *     workspace (size from pic_query_workspace) and keeps ownership of it;
 *     pic_free never frees caller memory.  Host allocations are limited to
 *     the handle and small metadata.
 *   - Work is enqueued on the caller's HIP stream (hipStream_t passed as
 *     void*; NULL = the null stream).  Calls that return data to the host
 *     synchronize that stream.
 *   - Every call returns a pic_status; pic_last_error() gives a message.
 *     Asynchronous device faults surface as PIC_EHIP at the next
 *     synchronizing call.  A handle is not thread-safe.
 */
#ifndef PIC_H
#define PIC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum pic_status {
    PIC_OK = 0,
    PIC_EINVAL = -1,     /* invalid argument or configuration               */
    PIC_ECAPACITY = -2,  /* a particle or child buffer would overflow       */
    PIC_EHIP = -3,       /* HIP runtime error (message has the HIP string)  */
    PIC_ENOCONV = -4,    /* field solve did not reach its tolerance         */
    PIC_ENAN = -5,       /* non-finite value detected                       */
    PIC_ESTATE = -6      /* call not valid in the handle's current state    */
} pic_status;

enum { PIC_MC = 0, PIC_EC = 1 };              /* field-gather scheme (Section 2) */
enum { PIC_F32 = 0, PIC_F64 = 1 };            /* particle-state precision        */
enum { PIC_FIXED_V = 0, PIC_RESISTOR = 1 };   /* cathode circuit (Sections 3-4)  */
enum { PIC_ABSORB = 0, PIC_REFLECT = 1 };     /* particle wall condition         */
enum { PIC_MGCG = 0, PIC_LEARNED = 1, PIC_CG = 2, PIC_DIRECT = 3 };
                                /* field solve: CG preconditioned by multigrid,
                                   by the learned network, or by nothing; or
                                   the direct sine-transform solve (needs a
                                   cathode covering the z = 0 row)         */

typedef struct pic_handle pic_handle;         /* opaque, library-owned */
typedef struct pic_ensemble pic_ensemble;     /* opaque, library-owned */

/* Problem definition.  Host arrays are read during pic_init only. */
typedef struct pic_config {
    int32_t nr, nz;             /* cells in r and z (>= 2)                        */
    double lr, lz;              /* domain r in [0, lr], z in [0, lz] (m)          */
    double dt;                  /* timestep (s)                                   */
    int32_t scheme;             /* PIC_MC or PIC_EC                               */
    int32_t precision;          /* PIC_F32 or PIC_F64 particle state              */
    double cathode_rmax;        /* z = 0 nodes with r < cathode_rmax are cathode;
                                   the rest of z = 0 is a Neumann block (Section 3) */
    int32_t circuit;            /* PIC_FIXED_V or PIC_RESISTOR                    */
    double v_fixed;             /* cathode voltage in PIC_FIXED_V mode (V)        */
    double v_ext, r_ext;        /* source voltage (V) and resistance (ohm)        */
    double gamma_i;             /* ion-induced secondary electron yield           */
    double p_gas, t_gas;        /* argon pressure (Pa), temperature (K)           */
    double e_exc, e_iz;         /* excitation, ionization thresholds (eV)         */
    const double *sigma;        /* host [4][n_table]: elastic, excitation,
                                   ionization from the ground state and from
                                   the metastable Ar* (Section 3's (1a)-(1d)),
                                   cross sections (m^2) at E_k = k * de_table eV */
    int32_t n_table;            /* >= 2                                           */
    double de_table;            /* eV                                             */
    const double *b_r, *b_z;    /* host nodal static magnetic field (T)           */
    double q[2], m[2], w[2];    /* charge (C), mass (kg), macro weight            */
    uint64_t seed;              /* Philox key                                     */
    uint32_t run;               /* ensemble index, selects the random stream      */
    int64_t capacity[2];        /* particle slots per species                     */
    int32_t sort_every;         /* steps between cell sorts (>= 1)                */
    int32_t poisson_mode;       /* PIC_MGCG, PIC_LEARNED (needs weights) or PIC_CG */
    double poisson_rtol;        /* FP64 relative residual target of each solve    */
    int32_t poisson_maxit;      /* cap on preconditioned CG iterations per solve  */
    int32_t wall_bc[3];         /* z = 0, z = lz, r = lr: PIC_ABSORB/PIC_REFLECT  */
    int32_t frozen_ions;        /* 1: ions are not pushed (test configurations)   */
    int32_t mcc_on, see_on;     /* enable collisions / secondary emission         */
    int32_t field_solve;        /* 0: keep phi fixed (push-only configurations)   */
    double extra_current;       /* synthetic current into the cathode (A)         */
    int32_t pc_batch;           /* training batch of the learned preconditioner;
                                   its buffers exist when pc_batch > 0 or
                                   poisson_mode = PIC_LEARNED (0..64)             */
    int32_t pc_maxit;           /* cap on learned-preconditioner iterations per
                                   solve before the multigrid fallback
                                   (0: poisson_maxit)                             */
    double gamma_e;             /* electron-induced secondary electron yield
                                   (Section 3: 0.1, independent of gamma_i)      */
    double n_meta;              /* static metastable Ar* density (m^-3), the
                                   target of process (1d) (Section 3: 2.5e17)    */
    double e_iz_meta;           /* ionization threshold from Ar* (eV, 4.20)      */
    int32_t deposit_fixed;      /* 1: FP64 state only; node charge summed as
                                   64-bit fixed point (tent weights rounded to
                                   multiples of 2^-42), so a step's result does
                                   not depend on the order of the deposit's
                                   additions: runs are bit-reproducible.  At
                                   most 2^21 particles may share a node.
                                   Single runs only (not ensembles).          */
    int32_t pc_pre;             /* learned preconditioner's first approximation
                                   x1 of A x = r: 0 a red-black Gauss-Seidel
                                   pair from zero, 1 one multigrid V-cycle
                                   (the multigrid preconditioner's)           */
} pic_config;

/* Initial particles of one species (host, FP64, absolute positions).
 * Velocities are taken as v^{n-1/2}.  ids must be unique per species. */
typedef struct pic_species_host {
    const double *r, *z, *vr, *vt, *vz;
    const uint32_t *id;
    int64_t n;
} pic_species_host;

/* Device view of one species' particle arrays (valid until the next call
 * that sorts: pic_step, pic_compact).  Positions are relative to the cell
 * (i, j), so r = (i + fr) * dr; velocities are v^{n-1/2} in (r, theta, z)
 * components.
 *   FP64 state (pos_bits = 0): key = j << 16 | i (-1: absorbed slot), fr/fz
 *     the in-cell fractions in [0,1) as doubles.
 *   FP32 state (pos_bits = 21, key_dev = NULL): fr_dev / fz_dev hold packed
 *     32-bit words pr = i << 21 | round(fr 2^21), pz = j << 21 |
 *     round(fz 2^21), pz = -1 for an absorbed slot (no key word is stored;
 *     cells are limited to 1024 per axis). */
typedef struct pic_particle_view {
    int32_t *key_dev;
    void *fr_dev, *fz_dev, *vr_dev, *vt_dev, *vz_dev;
    uint32_t *id_dev;
    int64_t count;              /* slots in use (live + not yet compacted)        */
    int64_t capacity;
    int32_t precision;
    int32_t pos_bits;           /* 0: key + fractions; 21: packed FP32 words      */
} pic_particle_view;

/* Device view of the node fields (FP64 unless stated). */
typedef struct pic_field_view {
    double *phi_dev;            /* phi^n = phi0 + V_c phi_L                        */
    double *phi0_dev;           /* solve with the cathode at 0 V                   */
    double *phi_l_dev;          /* unit-cathode Laplace solution                   */
    void *q_dev[2];             /* deposited node charge per species (C), in the
                                   particle precision                             */
    int64_t nodes;
    int32_t q_precision;
    double *phi0_prev_dev;      /* phi0 of the previous step                      */
} pic_field_view;

typedef struct pic_poisson_stats {
    int32_t iterations;         /* preconditioned CG iterations (all passes)     */
    int32_t outer;              /* FP64 refinement passes                         */
    double rel_res;             /* final ||b - K phi|| / ||b||, FP64              */
    int32_t fell_back;          /* learned preconditioner replaced by MG          */
    int32_t converged;
    int32_t pc_iterations;      /* of `iterations`, those with the learned
                                   preconditioner                                 */
} pic_poisson_stats;

/* Diagnostics (FP64).  ke/pz/dq refer to the last completed step. */
typedef struct pic_diag_out {
    int64_t step;
    double time;
    int64_t count[2];           /* live particles                                */
    double q_dep[2];            /* sum of deposited node charge                   */
    double q_expect[2];         /* q_s w_s N_s                                    */
    double ke[2];               /* 1/2 m w v^{n-1/2}.v^{n+1/2} summed            */
    double pz[2];               /* axial momentum at the new half step           */
    double w_field;             /* 1/2 sum_faces c (dphi)^2 of the current phi   */
    double dq_conv;             /* charge delivered to the cathode, last step    */
    double i_cathode;           /* dq_conv / dt                                   */
    double vc, qc, cap_c;       /* cathode voltage, charge, capacitance           */
    double n_peak[2];           /* max over nodes of Q_s / (q_s V_node)           */
    double phi_max;             /* max over nodes of phi                          */
    int64_t n_abs[2][5];        /* absorbed in the last step by wall code 1..4:
                                   cathode, Neumann block, outer r, anode        */
    int64_t n_cand, n_coll[4];  /* null-collision candidates; el, ex, iz, iz from
                                   the metastable                               */
    int64_t n_see;              /* ion-induced secondary electrons               */
    int64_t n_child[2];
    int64_t deposit_fallback;   /* wavefront chunks (256 particles) whose charge
                                   did not fit the LDS tile (global atomics)      */
    pic_poisson_stats poisson;  /* last field solve                               */
    int32_t flags;              /* bit 0 capacity, bit 1 child overflow, bit 2 NaN */
    int64_t n_see_e;            /* electron-induced secondary electrons          */
} pic_diag_out;

/* pic_step sorts the electrons every sort_every steps and the ions at
 * every PIC_ION_SORT_EVERY-th of those sorts: an ion moves ~1e-4 of a cell
 * per sort interval, so their order barely changes between sorts (the ions
 * created in between, appended at the end, and absorbed slots wait for the
 * next ion sort).  Ensembles sort both species at every sort step. */
#define PIC_ION_SORT_EVERY 4

/* Scalar state for checkpoint/resume.  A checkpoint is this state plus,
 * through the views, slots 0..count-1 of both species' arrays and phi0 and
 * phi0_prev (the field solve's warm start extrapolates from them).  To
 * resume, create a handle with the same configuration (pic_init with no
 * particles), write those arrays through its views, then call
 * pic_set_state.  With deposit_fixed = 1 and PIC_DIRECT the resumed run is
 * bit-identical to the uninterrupted one. */
typedef struct pic_scalar_state {
    int64_t step;
    double vc, qc;
    uint32_t next_id[2];
    int64_t count[2];
    int32_t sort_phase;         /* steps since the last cell sort (0..sort_every) */
    int32_t ion_sort_phase;     /* cell sorts since the ions were last sorted
                                   (0..PIC_ION_SORT_EVERY-1)                    */
} pic_scalar_state;

/* Per-phase device time accumulated from HIP events (ms), when enabled. */
typedef struct pic_timers {
    double push_ms, children_ms, sort_ms, poisson_ms, circuit_ms, field_ms;
    int64_t push_launches, sort_launches, poisson_solves;
} pic_timers;

/* Bytes of device workspace pic_init needs for cfg.  Errors: PIC_EINVAL. */
pic_status pic_query_workspace(const pic_config *cfg, int64_t *bytes);

/* Create a simulation in workspace_dev (>= the queried bytes, 256-byte
 * aligned).  init may be NULL (no particles) or point to two species.
 * Builds the collision tables, the multigrid hierarchy, phi_L and the
 * cathode capacitance, uploads and cell-sorts the particles, deposits and
 * solves the initial field.  Synchronizes the stream.
 * Errors: PIC_EINVAL (config), PIC_ECAPACITY (init larger than capacity),
 * PIC_EHIP, PIC_ENOCONV. */
pic_status pic_init(const pic_config *cfg, void *workspace_dev, int64_t workspace_bytes,
                    void *stream, const pic_species_host *init, pic_handle **out);

/* Advance nsteps (>= 0) explicit timesteps of the electrostatic PIC-MCC
 * cycle: field gather in the configured form (Section 2: EC-PIC edge fields
 * or MC-PIC nodal fields), Boris push and the R-Z rotation, particle walls
 * with ion- and electron-induced emission at the cathode (Section 3),
 * null-collision Monte Carlo collisions 1a-1d with the background Ar and Ar*
 * (Section 3), new particles, charge deposit, the field solve of Section 3's
 * charge-form Poisson equation and the external circuit (Section 3,
 * Table 1).  h: a handle from pic_init (not NULL).  Works on the handle's
 * stream; returns after the last step's work is enqueued and synchronizes
 * only where the field solve checks its residual.  A step that fails
 * leaves the state at that step (diagnostics name the cause).  Errors:
 * PIC_EINVAL (NULL handle, nsteps < 0), PIC_ECAPACITY (particle or child
 * buffers full), PIC_ENOCONV (field solve), PIC_EHIP. */
pic_status pic_step(pic_handle *h, int32_t nsteps);

/* Standalone field solve on the handle's grid: K phi = q with the cathode
 * nodes at v_cathode and the other Dirichlet nodes at 0.  phi_dev holds the
 * initial guess on entry (its Dirichlet entries are overwritten) and the
 * solution on exit; q_dev is node charge (C), FP64.  Uses the handle's
 * preconditioner mode, tolerance and iteration cap.  Synchronizes.
 * Errors: PIC_ENOCONV (stats still filled), PIC_EHIP. */
pic_status pic_poisson(pic_handle *h, const double *q_dev, double v_cathode, double *phi_dev,
                       pic_poisson_stats *stats);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * direct solve of pic_poisson (PIC_DIRECT) whose temporaries -- the FP64
 * residual, the two transform buffers and the residual norms -- live in a
 * static device array of the library instead of the handle's workspace.
 * Same arguments and results as pic_poisson: q_dev node charge (C, FP64),
 * phi_dev the initial guess on entry (Dirichlet entries overwritten) and
 * the solution on exit, both (nr+1)(nz+1) device doubles owned by the
 * caller; stats (host, nullable).  The handle must have been created with
 * poisson_mode = PIC_DIRECT (else PIC_ESTATE) and its device must be
 * current (else PIC_EINVAL).  The array holds 32 MiB per GPU (kept until
 * the process ends); a grid whose solve needs more -- (nr+1)(nz+1) + 2 Mp Np
 * doubles plus 24 KiB, Mp and Np the unknown rows and columns rounded up to
 * 32, e.g. 512 x 1024 cells fit, 1024 x 2048 do not -- gives PIC_EINVAL.
 * It calls no hipMalloc / hipFree and synchronizes the handle's stream.
 * Every call on a GPU shares that GPU's array: calls that overlap on one
 * GPU (other threads, other streams) race and must be serialized by the
 * caller.  Errors: PIC_ENOCONV (stats filled), PIC_EHIP. */
pic_status pic_poisson_static(pic_handle *h, const double *q_dev, double v_cathode,
                              double *phi_dev, pic_poisson_stats *stats);

/* out_dev = K phi_dev: the charge-form field operator of the solve (C per V;
 * Section 3's Gauss's law over each node's control volume) on unknown nodes,
 * 0 on Dirichlet nodes; phi_dev's Dirichlet entries are used as given.  FP64
 * node vectors.  Synchronizes. */
pic_status pic_apply_operator(pic_handle *h, const double *phi_dev, double *out_dev);

/* FP64 diagnostics of the current state into *out (host memory, not NULL):
 * counts, deposited and expected charge, kinetic energy and axial momentum,
 * field energy, the cathode's current, voltage and charge (the Section 4
 * observables: discharge current and voltage, peak densities, plasma
 * potential phi_max) and the step's event counts.  Synchronizes the
 * handle's stream.  Errors: PIC_EINVAL, PIC_EHIP. */
pic_status pic_diag(pic_handle *h, pic_diag_out *out);

/* Device views (synchronize to read counts). */
pic_status pic_particles(pic_handle *h, int32_t species, pic_particle_view *out);
pic_status pic_fields(pic_handle *h, pic_field_view *out);

/* Replace phi (host FP64 node array) and rebuild the gather fields; with
 * field_solve = 0 it stays fixed.  Synchronizes. */
pic_status pic_set_phi(pic_handle *h, const double *phi);

/* Cell-sort and compact both species now (drops absorbed slots). */
pic_status pic_compact(pic_handle *h);

/* ---- plasma diagnostics (Sections 4, 5 and 7) -------------------------------
 * Electron moments per cell (nearest grid point: cell (i, j) holds
 * i dr <= r < (i + 1) dr, j dz <= z < (j + 1) dz): count N, velocity sum S1
 * and sum of squared speeds S2, in FP64.  Cell maps: n = N w / V_cell with
 * V_cell = pi (r_{i+1}^2 - r_i^2) dz for both species; the electron
 * temperature T = m (S2 / N - |S1 / N|^2) / (3 e) in eV (cells with at least
 * two electrons; 0 elsewhere); the Debye length sqrt(eps0 T / (e n_e)) (m,
 * +inf where n_e or T is zero).  Section 4 compares with the cell size the
 * Debye length where the electron density is largest: lambda_d_peak is the
 * one of the first cell of largest n_e (j-major order).
 * Over the band of cells whose centre lies in [r0, r1) (Section 5 uses
 * 1.0 cm < r < 1.5 cm): per cell row the band densities (counts times w over
 * the band volume) and the band potential per node row (mean over the band
 * cells of the midpoint of each cell's lower edge), E_z = -d phi / dz per cell
 * row.  Sheath edge (Section 4: n_e = n_i / 2): the first cell row from the
 * cathode with n_e >= n_i / 2, interpolated linearly from the row below
 * between cell centres (0 if the first row qualifies, NaN if none).  Bulk
 * edge (E_z = 0): above the sheath edge, the first change of E_z from
 * negative to non-negative, interpolated likewise (NaN if none).  Region
 * temperatures (Section 5): count-weighted means of the band cells'
 * temperatures with the cell centre below the sheath edge (sheath), between
 * the edges (pre-sheath) and above the bulk edge (bulk); with no sheath edge
 * every band cell counts as sheath. */
typedef struct pic_plasma_out {
    double z_sheath, z_bulk;    /* m; NaN if not found                          */
    double te_region[3];        /* eV: sheath, pre-sheath, bulk                 */
    int64_t n_region[3];        /* electrons counted in each                    */
    double lambda_d_peak;       /* m, in the cell of largest n_e                */
    double n_e_peak;            /* m^-3, that cell's density                    */
    double te_peak;             /* eV, that cell's temperature                  */
    int32_t peak_cell[2];       /* (i, j) of that cell                          */
    int32_t band_cells[2];      /* the band's cells [i0, i1)                    */
} pic_plasma_out;

/* Compute the diagnostics of the current state (particles as they stand,
 * potential of the last step).  maps_host: NULL, or 4 nr nz doubles filled
 * with the cell maps n_e, n_i, T_e, lambda_D (cell (i, j) at j nr + i, one map
 * after the other).  Errors: PIC_EINVAL (r0 >= r1).  Synchronizes. */
pic_status pic_plasma_diagnostics(pic_handle *h, double r0, double r1, pic_plasma_out *out,
                                  double *maps_host);

/* Ion energy distribution at the cathode (Section 7): from the next step on,
 * every Ar+ absorbed by the cathode at radius r0 <= r < r1 adds one count to
 * bin floor(E / emax_ev * nbins), E = m_i |v|^2 / 2 in eV with the velocity of
 * its last push; E >= emax_ev counts in bin nbins.  nbins = 0 stops the
 * record.  Clears the counts.  Ensembles take the setting of their runs when
 * they are created.  Errors: PIC_EINVAL (nbins outside [0, 4096]; emax_ev <=
 * 0 or r0 >= r1 with nbins > 0).  Synchronizes. */
pic_status pic_ied_config(pic_handle *h, double emax_ev, int32_t nbins, double r0, double r1);

/* Copy the nbins + 1 counters to counts (host, ncounts = nbins + 1) and clear
 * them if reset != 0.  Errors: PIC_EINVAL (ncounts mismatch).  Synchronizes. */
pic_status pic_ied_read(pic_handle *h, uint64_t *counts, int32_t ncounts, int32_t reset);

/* Re-weighting (Section 5, removing particles and raising the weight when
 * the particle count grows large): keep the particles of both species whose
 * id is a multiple of keep_every, compact, and multiply both weights by
 * keep_every (the expected charge is unchanged).  The node charge follows at
 * the next step.  Not for runs that belong to an ensemble.  Errors:
 * PIC_EINVAL (keep_every outside [1, 1000]).  Synchronizes. */
pic_status pic_reweight(pic_handle *h, int32_t keep_every);

/* Scalar state (step, circuit, id counters, counts, sort phase) for
 * checkpointing (Section 2's timestep carries no other state between steps
 * than these, the particles and the potential).  pic_set_state also rebuilds
 * phi = phi0 + V_c phi_L and the gather fields from the handle's phi0 and the
 * restored V_c.  Errors: PIC_EINVAL (count above capacity, sort_phase outside
 * 0..sort_every, ion_sort_phase outside 0..PIC_ION_SORT_EVERY-1).  Both
 * synchronize. */
pic_status pic_get_state(const pic_handle *h, pic_scalar_state *out);
pic_status pic_set_state(pic_handle *h, const pic_scalar_state *in);

/* Per-phase HIP-event timing: on = 0 off, 1 every phase (particle kernel,
 * events and children, sort, field solve, circuit, field preparation), 2 the
 * particle kernel alone (two events per step instead of ten or more; the other
 * sums stay zero); other values give PIC_EINVAL.  pic_get_timers returns the
 * sums since the last reset and resets when reset != 0. */
pic_status pic_enable_timers(pic_handle *h, int32_t on);
pic_status pic_get_timers(pic_handle *h, pic_timers *out, int32_t reset);

/* ---- learned preconditioner of the field solve -----------------------------
 * The field solve of every step (Section 3's Gauss's law over the R-Z control
 * volumes, K phi = Q) runs conjugate gradients; PIC_LEARNED preconditions
 * them with a 4-level convolutional network f (15 3x3 convolutions with
 * ReLU, average pooling, nearest upsampling and additive skips; channels 16,
 * 16, 48, 80; inputs r1 / rms(r1) and i / 256), BF16 MFMA with FP32
 * accumulation, inside z = post(x1 + out_scale rms(r1) f(...), r): x1 a first
 * approximation of A x = r (pc_pre: one multigrid V-cycle, or a red-black
 * Gauss-Seidel pair from zero), r1 = r - A x1, post a black and a red
 * Gauss-Seidel sweep.  Because f is nonlinear the iteration is flexible CG
 * (Polak-Ribiere beta); when it reaches pc_maxit iterations without meeting
 * poisson_rtol, or stops reducing the residual, the solve continues from its
 * current iterate with multigrid-preconditioned CG (stats.fell_back = 1).
 * The set-up solves of pic_init always use multigrid.
 *
 * Parameters are one flat FP32 vector: for each convolution in order, its
 * weights [cout][cin][3][3] then its bias [cout]. */

/* Number of parameters of the network (196753). */
pic_status pic_pc_param_count(int64_t *n);

/* Load weights (host, n floats) and the output scale; resets Adam.
 * Errors: PIC_EINVAL (n mismatch), PIC_ESTATE (no preconditioner buffers:
 * pc_batch = 0 and poisson_mode != PIC_LEARNED).  Synchronizes. */
pic_status pic_pc_set_weights(pic_handle *h, const float *theta, int64_t n, double out_scale);
pic_status pic_pc_get_weights(pic_handle *h, float *theta, int64_t n, double *out_scale);

/* One Adam step (learning rate lr; lr = 0 computes loss and gradient only)
 * on `batch` pairs (q_dev: node charge in C, phi_dev: potential in V, FP64,
 * [batch][nodes]) with K phi = q and phi = 0 on every Dirichlet node, such
 * as (Q, phi0) of a step.  Loss: the mean over the pairs of
 * (1/2) e.A e / (phihat.A phihat), e = out_scale f(b / rho) - phi / rho on
 * unknown nodes, A = K / (2 pi eps0), b = A phi, rho = rms(b).  *loss gets
 * the loss before the update; grad (host, nullable, param_count floats)
 * the gradient.  1 <= batch <= pc_batch.  Synchronizes. */
pic_status pic_pc_train_step(pic_handle *h, const double *q_dev, const double *phi_dev,
                             int32_t batch, float lr, double *loss, float *grad);

/* z = the preconditioner applied to r (see above; 0 on Dirichlet nodes);
 * r_dev, z_dev FP64 node vectors in units of A = K / (2 pi eps0).  Uses the
 * multigrid level-0 buffers when pc_pre = 1.  Synchronizes. */
pic_status pic_pc_apply(pic_handle *h, const double *r_dev, double *z_dev);

/* Switch the preconditioner of later solves (PIC_LEARNED needs weights). */
pic_status pic_set_poisson_mode(pic_handle *h, int32_t mode);

/* ---- launch tuning ------------------------------------------------------------
 * The particle kernel's launch shape: total blocks, and the weight of an
 * electron against an ion when those blocks are split between the species
 * (electrons carry the collision test).  pic_autotune times candidate shapes
 * on the live simulation (block counts 256..8192 at the current weight, then
 * weights 1.0, 1.3, 1.7 at the best count), steps_per_trial (>= 1) steps
 * each, and keeps the fastest.  scratch_dev: a device buffer of the
 * caller's, at least pic_query_workspace bytes (scratch_bytes), into which
 * the workspace is copied before the trials and from which it is copied
 * back, with the host-side solver state, afterwards: the simulation is then
 * where it was before the call.  scratch_dev NULL: no copy, and the run
 * advances by 9 * steps_per_trial steps.  out (host, nullable) receives the
 * choice.  Synchronizes.  Errors: PIC_EINVAL (scratch too small,
 * steps_per_trial < 1), PIC_EHIP or a trial step's error.  The shape
 * changes no result beyond the summation order of the FP32 deposit.
 * pic_set_tuning applies a stored choice (e.g. from a run of the same size). */
typedef struct pic_tuning {
    int32_t push_blocks;        /* default 1024                                   */
    double push_e_weight;       /* default 1.3                                    */
    double push_ms;             /* autotune: mean particle-kernel time chosen     */
    int32_t trials;
    int32_t mg_one_level;       /* multigrid-preconditioned CG: 0 (default) runs
                                   pairs of the small grid levels above the
                                   single-workgroup coarse levels in one kernel
                                   each, and fuses the CG vector updates into
                                   the finest level's V-cycle kernels (p.q
                                   from dots of z, A z and q by the symmetry
                                   of A); 1 runs one kernel per level and
                                   separate CG kernels.  The two agree to FP32
                                   rounding.                                  */
    int32_t pass_graphs;        /* field-solve passes: 0 (default) launches their
                                   kernels directly; 1 captures a pass into a
                                   hipGraph on first use and replays it (on
                                   ROCm's graph launch, which enqueues node by
                                   node, the direct launches measured faster). */
} pic_tuning;

pic_status pic_autotune(pic_handle *h, int32_t steps_per_trial, void *scratch_dev,
                        int64_t scratch_bytes, pic_tuning *out);
pic_status pic_set_tuning(pic_handle *h, const pic_tuning *t);
pic_status pic_get_tuning(const pic_handle *h, pic_tuning *t);

/* ---- ensembles of independent discharges -----------------------------------
 * Many runs (each created by pic_init, with its own grid, particles,
 * secondary yield and circuit; Section 4's study varies the yield and the
 * external resistance) advance together: one step of every run is captured
 * once into a hipGraph and replayed each step as a single launch, with one
 * synchronization per step for the runs' status.  Each kernel of the step
 * (the cell sort of a sort step included) runs once for a batch of up to 64
 * runs, a block finding its run from block offsets, so the step is one
 * stream's work; nstreams must lie in 1..16 and is otherwise unused (kept so
 * that the signature stays stable).  Each field solve is multigrid-preconditioned and controlled on
 * the device: the step's graph holds its first pass, and while the status
 * shows a run short of poisson_rtol a captured one-pass graph runs again
 * (at most two more passes) for the runs not yet converged, so a run
 * advances exactly as pic_step would to within the solve tolerance.  The
 * runs must share sort_every and the state precision and have timers off;
 * creation cell-sorts every run so that all share one sort phase.  Runs are
 * not used through other calls while pic_ensemble_step runs.  The library
 * owns the streams, graphs and a small pinned status buffer; stream
 * (nullable) is where the graphs launch.  Errors of pic_ensemble_step name
 * the run: PIC_ECAPACITY, PIC_ENOCONV, PIC_EHIP.  Each run's descriptors
 * (of the batched solve and of its particle kernels) are written into its
 * own workspace at creation. */
pic_status pic_ensemble_create(pic_handle *const *runs, int32_t nruns, void *stream,
                               int32_t nstreams, pic_ensemble **out);
pic_status pic_ensemble_step(pic_ensemble *e, int32_t nsteps);
pic_status pic_ensemble_free(pic_ensemble *e);
const char *pic_ensemble_last_error(const pic_ensemble *e);

/* Destroy the handle: waits for its stream, releases what the library
 * allocated (pinned readback block, events, graphs); the caller's workspace
 * and stream stay the caller's.  NULL is accepted.  Lifecycle only (no
 * operation of the paper). */
pic_status pic_free(pic_handle *h);

/* Message of the last error on h (or of the last failed pic_init if h is
 * NULL).  Valid until the next call on the same handle. */
const char *pic_last_error(const pic_handle *h);

#ifdef __cplusplus
}
#endif
#endif /* PIC_H */
