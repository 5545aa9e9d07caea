/*
 * pic_oracle.h -- plain FP64 CPU oracle for one explicit electrostatic
 * 2D R-Z PIC-MCC timestep (test infrastructure only).
 *
 * This is the slow, obviously-correct reference that the GPU library is
 * checked against.  It shares no code with the GPU library.  Only the test
 * suite, the smoke check and the CPU-baseline leg of the benchmark may load it.
 *
 * What it follows (paper sections):
 *   Section 2   : MC-PIC gather (same linear stencil as the deposit) and
 *                 EC-PIC gather (edge-centred E, NGP along the component's
 *                 own direction, linear across it); nodal phi and rho.
 *   Section 3   : anode grounded at z = Z_max, cathode on z = 0 tied to an
 *                 external circuit, Neumann block beside it, Gauss's law on
 *                 the axis; absorbing z and outer-r walls, reflective axis;
 *                 constant ion-induced secondary yield, electrons emitted at
 *                 rest; MCC with elastic, excitation and ground-state
 *                 ionization collisions against a static argon background.
 *   Section 4   : external resistor between the source and the cathode.
 * Readings where the paper is silent (operator form, circuit law, collision
 * kinematics, random-number layout) are listed in the design notes and
 * restated at each function below.
 */
#ifndef PIC_ORACLE_H
#define PIC_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct orc_problem {
    int32_t nr, nz;            /* cells in r and z                          */
    double lr, lz, dt;         /* domain size (m) and timestep (s)          */
    int32_t scheme;            /* 0 = MC-PIC gather, 1 = EC-PIC gather      */
    double cathode_rmax;       /* z = 0 nodes with r < this are cathode     */
    int32_t circuit;           /* 0 = fixed cathode voltage, 1 = resistor   */
    double v_fixed, v_ext, r_ext;
    double gamma_i;            /* ion-induced secondary electron yield      */
    double p_gas, t_gas;       /* argon pressure (Pa) and temperature (K)   */
    double e_exc, e_iz;        /* excitation / ionization thresholds (eV)   */
    const double *sigma;       /* [4][n_table] cross sections (m^2): elastic,
                                  excitation, ionization from the ground
                                  state, ionization from the metastable    */
    int32_t n_table;
    double de_table;           /* table spacing (eV), E_k = k*de            */
    const double *b_r, *b_z;   /* nodal static B (T), index j*(nr+1)+i      */
    double q[2], m[2], w[2];   /* species 0 = electrons, 1 = Ar+            */
    uint64_t seed;
    uint32_t run;              /* ensemble member (random stream selector)  */
    int32_t wall_bc[3];        /* z=0, z=L, r=R: 0 absorb, 1 reflect        */
    int32_t frozen_ions, mcc_on, see_on, field_solve;
    double extra_current;      /* synthetic current into the cathode (A)    */
    double poisson_rtol;
    int32_t poisson_maxit;
    double gamma_e;            /* electron-induced secondary electron yield */
    double n_meta;             /* static Ar* (metastable) density (m^-3)    */
    double e_iz_meta;          /* ionization threshold from Ar* (eV)        */
    /* Ion energy distribution at the cathode (Section 7): when ied_hist is
     * not NULL, every Ar+ absorbed by the cathode with ied_r0 <= r' < ied_r1
     * adds one count to bin floor(E / ied_emax * ied_nbins) of ied_hist,
     * E = m |v|^2 / 2 (eV) with the velocity of its last push; energies at
     * or above ied_emax go to bin ied_nbins (ied_nbins + 1 counters). */
    double ied_emax, ied_r0, ied_r1;
    int32_t ied_nbins;
    uint64_t *ied_hist;
} orc_problem;

typedef struct orc_species {
    double *r, *z, *vr, *vt, *vz;
    uint32_t *id;
    int64_t n, cap;
} orc_species;

typedef struct orc_state {
    int64_t step;
    double vc, qc, cap_c;      /* cathode voltage, charge, capacitance     */
    uint32_t next_id[2];
} orc_state;

typedef struct orc_diag {
    double ke[2];              /* kinetic energy at the step's integer time */
    double pz[2];              /* axial momentum at the new half step       */
    double w_field;            /* field energy of the phi used by the push  */
    double q_dep[2];           /* sum of deposited node charge per species  */
    double dq_conv;            /* charge delivered to the cathode this step */
    double qc0;                /* induced cathode charge of phi0            */
    int64_t n_abs[2][5];       /* absorbed per species by wall code 1..4    */
    int64_t n_cand, n_coll[4]; /* null-collision candidates; el, ex, iz,
                                  iz from Ar*                              */
    int64_t n_see;             /* ion-induced secondary electrons          */
    int64_t n_child[2];
    int64_t poisson_iters;
    double poisson_res;
    double n_peak[2];          /* max over nodes of Q_s / (q_s V_node) after the deposit */
    double phi_max;            /* max over nodes of the new phi             */
    double i_cathode;          /* dq_conv / dt                              */
    int64_t n_see_e;           /* electron-induced secondary electrons      */
} orc_diag;

/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11). */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* Field-solve pieces (nodes ordered j*(nr+1)+i). */
int  orc_node_kind(const orc_problem *p, int i, int j);            /* 0 unknown, 1 cathode, 2 grounded */
void orc_couplings(const orc_problem *p, double *c_east, double *c_north);
void orc_apply_k_full(const orc_problem *p, const double *phi, double *out);
int  orc_solve(const orc_problem *p, const double *q_node, double v_cathode,
               double *phi, double rtol, int maxit, int64_t *iters, double *rel_res);
double orc_field_energy(const orc_problem *p, const double *phi);
void orc_nodal_e(const orc_problem *p, const double *phi, double *er, double *ez);
/* Node volumes of the density diagnostic: the volume a tent weight of node
 * (i,j) integrates to over the cylinder (linear-in-r weighting). */
void orc_node_volumes(const orc_problem *p, double *vol);
/* Circuit pieces: capacitance sum over cathode nodes of (K phi_L), and the
 * induced cathode charge sum over cathode nodes of (K phi0 - Q). */
double orc_capacitance(const orc_problem *p, const double *phi_l);
double orc_induced_charge(const orc_problem *p, const double *phi0, const double *q_node);

/* Particle-grid pieces. */
void orc_deposit(const orc_problem *p, const double *r, const double *z, int64_t n,
                 double qw, double *q_node);
void orc_gather(const orc_problem *p, const double *phi, const double *r, const double *z,
                int64_t n, double *er, double *ez, double *br, double *bz);

/* Collision tables: nu[4][n_table] (1/s), returns nu_max; *t_null = floor(P_null 2^32). */
double orc_nu_tables(const orc_problem *p, double *nu, uint64_t *t_null);

/* The null-collision decision of one electron with velocity v (after the
 * push) at step `step`: -2 not a candidate, -1 null collision, 0 elastic,
 * 1 excitation, 2 ionization from the ground state, 3 from the metastable.  *margin (nullable) receives the smallest
 * relative distance of the floating-point comparisons that decide the
 * process: |R - cumulative nu_k| / nu_max and |E - E_threshold| / E_threshold
 * (0 when the electron is not a candidate: that test is an integer one). */
int orc_mcc_select(const orc_problem *p, const double *nu, double numax, uint64_t t_null,
                   uint32_t id, int64_t step, double vr, double vt, double vz, double *margin);
/* orc_mcc_select for n electrons (codes[k], margins[k] nullable). */
void orc_mcc_select_many(const orc_problem *p, int64_t step, int64_t n, const uint32_t *id,
                         const double *vr, const double *vt, const double *vz, int32_t *codes,
                         double *margins);

/* Whole-run drivers. phi, phi0, phi_l and q_node[2] are node arrays. */
/* Threads the particle loops use: 1 in the serial build, the OpenMP team
 * size in the multi-core timing build. */
int orc_thread_count(void);

int orc_init(const orc_problem *p, orc_species sp[2], orc_state *st,
             double *phi, double *phi0, double *phi_l, double *q_e, double *q_i);
int orc_step(const orc_problem *p, orc_species sp[2], orc_state *st,
             double *phi, double *phi0, const double *phi_l, double *q_e, double *q_i,
             orc_diag *d);

#ifdef __cplusplus
}
#endif
#endif
