// Internal declarations of libpic.so (device structs, helpers, launchers).
//
// Layout in HBM (all carved from the caller's workspace):
//   particles, per species, structure of arrays with `cap` slots, twice
//   (ping-pong for the cell sort): key int32 (j << 16 | i, -1 = absorbed),
//   fr, fz, vr, vt, vz in the state precision T, id uint32;
//   node fields: one 4-vector per node (T4 = float4 / double4) holding the
//   gather inputs (E_r, E_z, B_r, B_z); for EC-PIC the E entries are the
//   edge values E_r(i+1/2, j) and E_z(i, j+1/2) of Section 2's staggering;
//   node charge per species in T; phi, phi0, phi_L and the FP64 operator in
//   FP64; the FP32 multigrid hierarchy.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/pic.h"

namespace pic {

constexpr int PUSH_THREADS = 256;
constexpr int PUSH_PPT = 4;                        // particles per thread per chunk
constexpr int PUSH_CHUNK = PUSH_THREADS * PUSH_PPT;
constexpr int LDS_NODES = 4096;                    // deposit tiles of a block (nodes)
constexpr int MAX_LEVELS = 16;
constexpr int MG_TAIL_LDS_MAX = 128 * 1024;        // dynamic LDS of the coarse-level kernels
constexpr int MG_TAIL_NODES_MAX = 4096;            // nodes of the first level of that kernel
constexpr int MAX_PCG = 512;
constexpr int MAX_BATCH = 64;
// Sums that hundreds of blocks finishing together accumulate with FP64
// atomics are spread over ACC_SLOTS partial sums, a block adding to slot
// (block mod ACC_SLOTS), each slot on its own 64-byte line: atomics of every
// block to one address serialize and hold the kernel's completion by
// microseconds.
constexpr int ACC_SLOTS = 16, ACC_STRIDE = 8;

enum : int32_t { FLAG_CAPACITY = 1, FLAG_CHILD_OVERFLOW = 2, FLAG_NAN = 4, FLAG_NOCONV = 8 };

template <typename T> struct Vec4;
template <> struct Vec4<float> { using type = float4; };
template <> struct Vec4<double> { using type = double4; };

// Device-resident scalar state of one simulation.
struct DevScalars {
    // read back together (one copy) after each field-solve pass
    double res_rr, res_bb;      // FP64 residual and rhs norms^2
    double res_rr0;             // residual norm^2 at the start of the pass
    int32_t flags;
    int32_t pad_;
    int64_t count[2];           // slots in use per species
    int64_t step;
    uint32_t next_id[2];
    int32_t n_child;            // children recorded this step (all species)
    int32_t n_mcc_q, n_see_q;   // event-queue lengths of the step
    int32_t n_child_s[2];       // children per new-particle species
    double dq_conv;             // charge into the cathode this step
    double ke[2], pz[2];
    unsigned long long n_abs[2][5];
    unsigned long long n_cand, n_coll[4], n_see, n_see_e;
    unsigned long long deposit_fallback;
    double vc, qc, cap_c, qc0;
    // sort
    int64_t sort_total[2];
    // field solve accumulators
    double pcg_rz[MAX_PCG + 2], pcg_pq[MAX_PCG + 2], pcg_rr[MAX_PCG + 2];
    double pcg_zq[MAX_PCG + 2];     // z_k . q_{k-1} (flexible CG)
    double pcg_ss[MAX_PCG + 2];     // sum r^2 of each learned-preconditioner input
    // device-controlled solve of a captured step: done flag (gates the pass
    // kernels), passes and iterations run
    int32_t solve_done, solve_passes, solve_iters;
    int32_t post_done;          // ensembles: circuit and gather fields done this step
    // a single run's FP64 residual norms^2 (||r||^2, ||b||^2) in ACC_SLOTS
    // slots each, summed by their readers (the cast kernel, the host)
    double res_slots[2 * ACC_SLOTS * ACC_STRIDE];
};
constexpr int RES_SLOT_WORDS = 2 * ACC_SLOTS * ACC_STRIDE;

// Particle arrays of one species (structure of arrays).
//
// Positions are kept relative to the particle's cell.  FP64 state: key =
// j << 16 | i (-1 once absorbed) and the in-cell fractions fr, fz in [0, 1)
// as FP64.  FP32 state packs the cell into the fraction words, so a particle
// carries no key word: pr = i << 21 | round(fr 2^21) and pz = j << 21 |
// round(fz 2^21) (-1 once absorbed), stored in the fr / fz arrays, key unused.
// Both words are non-negative for live particles (cells < 1024 per axis),
// and the fractions resolve 2^-21 of a cell.
template <typename T>
struct SpeciesDev {
    int32_t *key;
    T *fr, *fz, *vr, *vt, *vz;
    uint32_t *id;
};

constexpr int POS_BITS = 21;                       // fraction bits of a packed word
constexpr int POS_MAX_CELLS = 1 << (31 - POS_BITS); // cells per axis with FP32 state
constexpr uint32_t POS_MASK = (1u << POS_BITS) - 1u;

// packed word of cell index c and in-cell fraction f in [0, 1), rounded to
// nearest (the top 2^-22 of a cell rounds down, never into the next cell)
__device__ __forceinline__ uint32_t pos_pack(int c, float f)
{
    const uint32_t q = (uint32_t)rintf(f * (float)(1u << POS_BITS));
    return ((uint32_t)c << POS_BITS) | min(q, POS_MASK);
}
__device__ __forceinline__ int pos_cell(uint32_t w) { return (int)(w >> POS_BITS); }
__device__ __forceinline__ float pos_frac(uint32_t w)
{
    return (float)(w & POS_MASK) * (1.0f / (float)(1u << POS_BITS));
}

// An in-cell offset as the state stores it: FP32 rounds to the packed
// fraction, FP64 keeps it.
__device__ __forceinline__ float pos_round(float f)
{
    const float q = fminf(rintf(f * (float)(1u << POS_BITS)), (float)POS_MASK);
    return fmaxf(q, 0.0f) * (1.0f / (float)(1u << POS_BITS));
}
__device__ __forceinline__ double pos_round(double f) { return f; }

// A step's displacement (cells) rounded to a whole number of position
// quanta (2^-21 cell), down after adding d16 / 65536 of a quantum: the
// rounding is exact on average.  The FP32 state holds the offset on the
// quantum grid, so the new offset (old + rounded displacement) is exact; had
// the sum been rounded to nearest instead, a particle of steady velocity
// would lose the same fraction of a quantum every step, and one that moves
// less than half a quantum per step would never move.
__device__ __forceinline__ float step_round(float d, uint32_t d16)
{
    const float x = fmaf(d, (float)(1u << POS_BITS), (float)d16 * (1.0f / 65536.0f));
    return floorf(x) * (1.0f / (float)(1u << POS_BITS));
}

// Dither bits of one particle slot and step, 16 per axis: for a fixed slot
// the top bits of a Weyl sequence in the step, offset per slot and run
// (increments 0x9E3779B9 and 0x6A09E667, the fractional parts of the golden
// ratio and of sqrt 2 in 32-bit fixed point), so over consecutive steps a
// particle's dither visits [0, 1) evenly and its rounding errors cancel.
__device__ __forceinline__ uint32_t dither_bits(uint32_t slot, uint32_t step, uint32_t word)
{
    const uint32_t r = slot * 0x85EBCA6Bu + step * 0x9E3779B9u + word * 0xC2B2AE35u;
    const uint32_t z = slot * 0x27D4EB2Fu + step * 0x6A09E667u + word * 0x165667B1u;
    return (r >> 16) | (z & 0xFFFF0000u);
}

// Position of slot p: returns the key j << 16 | i (-1 if absorbed) and the
// fractions (also of an absorbed slot: its last cell and offsets).
template <typename T>
__device__ __forceinline__ int load_pos(const SpeciesDev<T> &S, int64_t p, T &fr, T &fz, int &i)
{
    if constexpr (sizeof(T) == 4) {
        const uint32_t wr = ((const uint32_t *)S.fr)[p];
        const int32_t wz = ((const int32_t *)S.fz)[p];
        i = pos_cell(wr);
        fr = pos_frac(wr);
        fz = wz >= 0 ? pos_frac((uint32_t)wz) : (T)0;
        return wz >= 0 ? (pos_cell((uint32_t)wz) << 16) | i : -1;
    } else {
        const int k = S.key[p];
        fr = S.fr[p];
        fz = S.fz[p];
        i = k >= 0 ? (k & 0xffff) : 0;
        return k;
    }
}

// Store the position of slot p: live in cell (i, j), or absorbed (alive =
// false; FP32 keeps i and fr in the pr word).
template <typename T>
__device__ __forceinline__ void store_pos(const SpeciesDev<T> &S, int64_t p, bool alive, int i,
                                          int j, T fr, T fz)
{
    if constexpr (sizeof(T) == 4) {
        ((uint32_t *)S.fr)[p] = pos_pack(min(max(i, 0), POS_MAX_CELLS - 1), fr);
        ((int32_t *)S.fz)[p] = alive ? (int32_t)pos_pack(j, fz) : -1;
    } else {
        S.key[p] = alive ? ((j << 16) | i) : -1;
        S.fr[p] = fr;
        S.fz[p] = fz;
    }
}

// Word that is negative exactly for absorbed slots (sort, live counts).
template <typename T>
__host__ __device__ __forceinline__ const int32_t *live_words(const SpeciesDev<T> &S)
{
    if constexpr (sizeof(T) == 4) return (const int32_t *)S.fz;
    else return S.key;
}

// A particle created during the push (ionization products, emitted
// secondaries).  skey orders children by (parent species, parent id, kind).
template <typename T>
struct Child {
    unsigned long long skey;
    int32_t species;
    int32_t key;
    T fr, fz, vr, vt, vz;
};

// Constants of the rare branches of the particle kernel (collisions,
// emission, new particles), kept in device memory so that the kernel reads
// them where they are used instead of holding them in scalar registers.
template <typename T>
struct PushCold {
    Child<T> *child;
    int32_t child_cap;
    const T *nu;                // [4][n_table] collision frequencies (1/s)
    int32_t n_table;
    T inv_de, numax;
    unsigned long long t_see[2];  // emission thresholds per absorbed species
    T e_of_v2;                  // m_e / (2 e): eV per (m/s)^2
    T v2_of_e;                  // 2 e / m_e
    T two_m_over_M;             // elastic energy-loss factor 2 m_e / M
    T e_exc, e_iz, e_iz_meta;   // thresholds (eV): excitation, ionization (1c), (1d)
    T sig_ion;                  // new-ion thermal speed sqrt(kT/M)
    double qw64[2];             // q w in FP64 for the cathode tally
    int32_t wall_bc[3];
    T cathode_rmax;
};

template <typename T>
struct PushParams {
    SpeciesDev<T> sp[2];
    const typename Vec4<T>::type *node;
    T *q[2];
    DevScalars *sc;
    const PushCold<T> *cold;
    int2 *mcc_q, *see_q;        // event queues (slot, aux)
    int32_t ev_cap;
    unsigned long long t_null;
    int32_t nr, nz;
    T dr, inv_dr, inv_dz, dt;
    T hqm[2];                   // q dt / (2 m)
    T qw[2];                    // q w (C per macroparticle)
    double mw[2];               // m w (kg per macroparticle), diagnostics
    int32_t frozen_ions, mcc_on;
    int32_t emit[2];            // absorbed particles of the species may emit
    int32_t any_reflect;        // some wall reflects (test configurations)
    int32_t deposit_only;       // 1: only deposit the current positions
    uint32_t key0, key1, run;
    int32_t nblk_e;             // blocks [0, nblk_e) push electrons, the rest ions
    int32_t fixed_q;            // 1: fixed-point node charge (FP64 state)
    int32_t ied_on;             // 1: ions absorbed by the cathode are queued for the
                                //    energy record even without emission
};

template <typename T>
struct EventParams {
    SpeciesDev<T> sp[2];
    const PushCold<T> *cold;
    DevScalars *sc;
    const int2 *mcc_q, *see_q;
    int32_t ev_cap;
    int32_t nr;
    uint32_t key0, key1, run;
    // cathode ion-energy record (ied_hist == nullptr: off): ions absorbed with
    // ied_r0 <= r < ied_r1 count in bin floor(E / ied_emax * ied_nbins),
    // E = ied_m |v|^2 / 2 (eV), the last bin taking E >= ied_emax
    unsigned long long *ied_hist;
    double ied_emax, ied_r0, ied_r1, ied_m, dr;
    int32_t ied_nbins;
};

template <typename T>
struct ChildParams {
    SpeciesDev<T> sp[2];
    int64_t cap[2];
    T *q[2];
    T qw[2];
    DevScalars *sc;
    const Child<T> *child;
    int32_t child_cap;
    int32_t nr;
    int32_t fixed_q;            // 1: fixed-point node charge (FP64 state)
    double qw64[2];             // q w in FP64: the cathode charge of the step
};

// The cell sort of one species of a run: from the current buffer (src) into
// the other (dst), with the run's bin counts and tile sums (shared by its two
// species, which sort one after the other).
template <typename T>
struct SortJob {
    SpeciesDev<T> src, dst;
    DevScalars *sc;
    int32_t *hist, *block_sums;
    int32_t nr, nbins;
};

// A run's particle-kernel parameters for one pair of current particle
// buffers; an ensemble keeps the four pairs in each run's workspace.
template <typename T>
struct RunParticles {
    PushParams<T> push;
    EventParams<T> ev;
    ChildParams<T> ch;
    SortJob<T> sort[2];         // per species
};

// The sort of one species in every run of a batch, one launch per kernel:
// job[r] points at run r's two SortJobs; off holds each run's first block
// (set per kernel by the launcher), nbins each run's bin count.
template <typename T>
struct SortBatch {
    const SortJob<T> *job[MAX_BATCH];
    int32_t off[MAX_BATCH + 1];
    int32_t nbins[MAX_BATCH];
    int32_t nruns, species;
};

// One launch of a particle kernel for up to MAX_BATCH runs: each run's
// descriptor, its first block (a block finds its run by binary search over
// off) and, for the push, its electron blocks (aux).
template <typename T>
struct PartBatch {
    const RunParticles<T> *p[MAX_BATCH];
    int32_t off[MAX_BATCH + 1];
    int32_t aux[MAX_BATCH];
    int32_t nruns;
};

// ---------------------------------------------------------------- Philox --
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 32x32->64 products of counter words 0 and 2 with the round multipliers,
// high halves xored with words 1, 3 and the key, key bumped by the Weyl
// increments between rounds.
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // one 32 x 32 -> 64-bit product per multiplier (a single
        // v_mad_u64_u32, instead of separate high and low multiplies)
        const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// Counter layout of every draw: (particle id, run << 8 | species << 4 |
// purpose, step, 0).  Purposes: 0 collision (candidate, process, direction),
// 1 ionization extras (energy split, ejected direction), 2 new-ion velocity,
// 3 secondary emission.
enum : uint32_t { PURPOSE_MCC = 0, PURPOSE_IZ = 1, PURPOSE_ION = 2, PURPOSE_SEE = 3 };

template <typename T>
__device__ __forceinline__ T u24(uint32_t u) { return (T)(u >> 8) * (T)(1.0 / 16777216.0); }
// Uniform on (0,1) for log(): midpoint of a 23-bit cell, exact in binary32.
template <typename T>
__device__ __forceinline__ T u_open(uint32_t u) { return ((T)(u >> 9) + (T)0.5) * (T)(1.0 / 8388608.0); }

__device__ __forceinline__ void sincos_2pi(float u, float *s, float *c) { sincospif(2.0f * u, s, c); }
__device__ __forceinline__ void sincos_2pi(double u, double *s, double *c) { sincospi(2.0 * u, s, c); }

// ----------------------------------------------------------- wave helpers --
// Column i and row j of node n of a grid with ld nodes per row.  Node
// indices stay below 2^31, so a 32-bit division does (a 64-bit one is an
// expensive software routine on the GPU).
__device__ __forceinline__ void node_ij(int64_t n, int ld, int &i, int &j)
{
    const uint32_t u = (uint32_t)n;
    j = (int)(u / (uint32_t)ld);
    i = (int)(u - (uint32_t)j * (uint32_t)ld);
}

// A solve's gate flag (kernels return at once when it is set and nonzero),
// read with a vector load from a flag that is always there (a zero one when
// the solve has none): it then completes in order with the data loads a
// kernel issues after it and is waited for only where it is tested, whereas
// a scalar load, or a branch around the load, waits for it up front.
static __device__ int32_t gate_never;
__device__ __forceinline__ int32_t gate_load(const int32_t *gate)
{
    return __hip_atomic_load(gate ? gate : &gate_never, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
}

// Order the LDS accesses of one wavefront's lanes before and after this point
// (the lanes of a wavefront share the instruction stream; this keeps the
// compiler from moving LDS accesses across it).
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ int wave_min(int v)
{
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ int wave_max(int v)
{
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ double wave_sum(double v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Fixed-point node charge: a tent weight w (|w| < 512) rounded to the
// nearest multiple of 2^-QFIX_BITS, as an integer.  w 2^42 + 1.5 2^52 lies in
// [2^52, 2^53), where doubles are spaced by 1, so the one rounding of the
// fused multiply-add leaves round(w 2^42) in the low mantissa bits.
constexpr int QFIX_BITS = 42;
__device__ __forceinline__ long long to_fixed(double w)
{
    const double m = __fma_rn(w, 0x1p42, 0x1.8p52);
    return __double_as_longlong(m) - 0x4338000000000000LL;
}

// Global float/double atomic add using the hardware instruction (the
// workspace is coarse-grained device memory).
__device__ __forceinline__ void atomic_add_dev(float *p, float v) { unsafeAtomicAdd(p, v); }
__device__ __forceinline__ void atomic_add_dev(double *p, double v) { unsafeAtomicAdd(p, v); }

// --------------------------------------------------------------- launchers --
// particles.hip
template <typename T>
void launch_push(const PushParams<T> &p, int scheme, int nblocks, hipStream_t s);
template <typename T>
void launch_push_b(const PartBatch<T> &b, int scheme, hipStream_t s);
template <typename T>
void launch_begin_b(const PartBatch<T> &b, hipStream_t s);
template <typename T>
void launch_events_b(const PartBatch<T> &b, hipStream_t s);
template <typename T>
void launch_children_b(const PartBatch<T> &b, hipStream_t s);
template <typename T>
void launch_finalize_b(const PartBatch<T> &b, hipStream_t s);
// blocks per run of the batched begin, event and child kernels
int begin_b_blocks(int64_t nodes, int elem_bytes);
constexpr int EVENTS_B_BLOCKS = 128;
int children_b_blocks(int32_t child_cap);
template <typename T>
void launch_events(const EventParams<T> &p, hipStream_t s);
template <typename T>
void launch_children(const ChildParams<T> &p, hipStream_t s);
void launch_finalize_step(DevScalars *sc, const int64_t cap[2], const double qw64[2],
                          hipStream_t s);
// fixed-point node charge (64-bit integers in place) to FP64 charge
void launch_q_from_fixed(void *q0, void *q1, int64_t nodes, const double qw64[2], hipStream_t s);

// diagnostics.hip: plasma diagnostics of Sections 4, 5 and 7
constexpr int IED_MAX_BINS = 4096;
struct PlasmaDev {
    double *mom[2];             // per species 5 x ncell: count, sum vr, vt, vz, |v|^2
    double *maps;               // 4 x ncell: n_e, n_i, T_e, lambda_D
    double *prof;               // 3 x (nz + 1): band n_e, n_i, phi
    void *out;                  // PlasmaOut
    unsigned long long *ied;    // IED_MAX_BINS + 1 counters
};
struct PlasmaOut {
    double z_sheath, z_bulk;
    double te_region[3];
    double n_region[3];
    double lambda_d_peak, n_e_peak, te_peak;
    int32_t peak_i, peak_j;
};
struct PlasmaArgs {
    int32_t nr, nz;
    double dr, dz;
    double w[2], m_e;
    int32_t ib0, ib1;           // band cells [ib0, ib1)
};
template <typename T>
void launch_cell_moments(const SpeciesDev<T> &S, int64_t n, int nr, int nz, double *mom,
                         hipStream_t s);
void launch_plasma(const PlasmaDev &D, const PlasmaArgs &A, const double *phi, hipStream_t s);
template <typename T>
void launch_reweight(const SpeciesDev<T> &S, int64_t n, uint32_t keep_every, hipStream_t s);
void launch_begin_step(DevScalars *sc, void *q0, void *q1, int64_t nodes, int elem_bytes,
                       hipStream_t s);
template <typename T>
void launch_load(SpeciesDev<T> sp, int64_t offset, const double *r, const double *z,
                 const double *vr, const double *vt, const double *vz, const uint32_t *id,
                 int64_t n, int32_t nr, int32_t nz, double dr, double dz, hipStream_t s);

// sort.hip
// cap[r]: run r's capacity of the species (sets its blocks)
template <typename T>
void launch_sort_b(SortBatch<T> b, const int64_t *cap, hipStream_t s);
template <typename T>
void launch_sort(SpeciesDev<T> src, SpeciesDev<T> dst, DevScalars *sc, int species,
                 int32_t *hist, int32_t *block_sums, int32_t nr, int32_t nz, int64_t cap,
                 hipStream_t s);

// mg.hip: matrix-free multigrid levels (couplings / (2 pi eps0))
struct MGLevel {
    int32_t nr, nz;
    int32_t cath;               // nodes i < cath of row j = 0 are cathode (Dirichlet)
    float dz, dr2dz;            // dz and dr^2 / dz of the level
    float *b;                   // right-hand side
    float *xd;                  // correction after pre-smoothing (down pass)
    float *xu;                  // correction after post-smoothing (up pass)
    const int32_t *gate;        // when set and nonzero, the kernels return at once
};

// Matrix-free operator of a level, divided by 2 pi eps0: east face (i+1/2, j)
// coupling (i + 1/2) hz_j with hz_j = dz (dz/2 on the z walls); north face
// (i, j+1/2) coupling g_i dr^2 / dz with g_0 = 1/8, g_i = i, g_nr = nr/2 - 1/8.
// Unknown nodes exclude the anode row, the outer column and the cathode.
__device__ __forceinline__ bool mg_in(const MGLevel &L, int i, int j)
{
    return i >= 0 && j >= 0 && i <= L.nr && j <= L.nz;
}
__device__ __forceinline__ bool mg_unknown(const MGLevel &L, int i, int j)
{
    return i < L.nr && j < L.nz && !(j == 0 && i < L.cath);
}
// couplings of an unknown node (i, j) of a level with nr x nz cells: west,
// east, south, north (0 if absent); every term is computed and the absent
// ones selected away, so the code has no branches
__device__ __forceinline__ void mg_coup_v(int nr, int nz, float dz, float dr2dz, int i, int j,
                                          float &w, float &e, float &s, float &n)
{
    const float hz = (j == 0 || j == nz) ? 0.5f * dz : dz;
    const float g = (i == 0) ? 0.125f : ((i == nr) ? 0.5f * (float)nr - 0.125f : (float)i);
    const float an = g * dr2dz;
    const float aw = ((float)(i - 1) + 0.5f) * hz;
    w = (i > 0) ? aw : 0.0f;
    e = ((float)i + 0.5f) * hz;
    s = (j > 0) ? an : 0.0f;
    n = an;
}
__device__ __forceinline__ void mg_coup(const MGLevel &L, int i, int j, float &w, float &e,
                                        float &s, float &n)
{
    mg_coup_v(L.nr, L.nz, L.dz, L.dr2dz, i, j, w, e, s, n);
}

// bilinear prolongation from the coarse values around fine node (i, j):
// c0 at (i/2, j/2), c1 east of it, c2 north, c3 north-east (c1..c3 are read
// only where the parity of i, j needs them)
__device__ __forceinline__ float mg_prolong_sel(bool oi, bool oj, float c0, float c1, float c2,
                                                float c3)
{
    return (oi && oj) ? 0.25f * (c0 + c1 + c2 + c3)
           : oi       ? 0.5f * (c0 + c1)
           : oj       ? 0.5f * (c0 + c2)
                      : c0;
}

struct MGTail {
    MGLevel L[MAX_LEVELS];
    int32_t first, last;        // levels handled inside one workgroup
    int32_t tmp_size;           // nodes of level `first`
    int32_t offx[MAX_LEVELS];   // LDS float offsets of each level's x and b
    int32_t offb[MAX_LEVELS];
    const float *inv;           // dense inverse on the coarsest unknowns
    const int32_t *map;         // unknown index -> node index (coarsest level)
    int32_t ninv;
};

struct MGHier {
    MGLevel lv[MAX_LEVELS];
    int32_t nlevels;
    MGTail tail;
    int32_t tail_lds_bytes;
};

// lv[0].xu = M lv[0].b; two_level: pairs of small grid levels in one kernel
void launch_mg_vcycle(const MGHier &H, double *dot, hipStream_t s, bool two_level);
// p = z + beta p_prev, q = A p, pq[0] += p.q (pq = &pcg_pq[k]); beta from
// rz (Fletcher-Reeves) or, when zq is given, Polak-Ribiere (flexible CG)
void launch_cg_matvec(const MGHier &H, const float *z, const float *pp, float *pc, float *q,
                      const double *rz, int k, double *pq, const double *zq, hipStream_t s);
void launch_cg_update(const MGHier &H, const float *p, const float *q, float *e, float *r,
                      const double *rz, const double *pq, double *rr, hipStream_t s);
int mg_tail_setup(MGHier &H);

// Preconditioned CG fused into the finest level's V-cycle kernels.  The "up"
// kernel of iteration k also forms w_k = A z_k and the dots r_k.z_k, z_k.w_k,
// z_k.q_{k-1}; the next V-cycle's "down" kernel first applies the update of
// iteration k on its tile (p_k = z_k + beta p_{k-1}, q_k = w_k + beta q_{k-1}
// = A p_k, p_k.q_k = z.w + 2 beta z.q_{k-1} + beta^2 p_{k-1}.q_{k-1} by the
// symmetry of A, alpha, e += alpha p_k, r_{k+1} = r_k - alpha q_k) and smooths
// r_{k+1}.  r and q are double-buffered: a tile reads its halo's old values
// while its owned nodes get the new ones.
// Each dot product is accumulated in CG_SLOTS partial sums (ACC_SLOTS).
// Iteration k's quantity m (0 r.z, 1 z.w, 2 z.q_{k-1}, 3 ||r_{k+1}||^2) sits
// at acc + cg_acc_at(k, m, slot).
constexpr int CG_SLOTS = ACC_SLOTS, CG_SLOT_STRIDE = ACC_STRIDE;
constexpr int CG_ACC_PER_ITER = 4 * CG_SLOTS * CG_SLOT_STRIDE;
__host__ __device__ constexpr int cg_acc_at(int k, int m, int slot)
{
    return (k * 4 + m) * CG_SLOTS * CG_SLOT_STRIDE + slot * CG_SLOT_STRIDE;
}
struct CgVecs {
    float *r[2], *q[2], *w, *p, *e;
    double *acc;                        // slotted dots, cleared per pass
    double *pq;                         // p_k.q_k per iteration
};
// z = M r[k & 1] into lv[0].xu, with w and the dots; for k > 0 the down
// kernel first applies update k - 1 (r[k & 1] = r_k from r[(k - 1) & 1])
void launch_mg_vcycle_cg(const MGHier &H, const CgVecs &v, int k, hipStream_t s, bool two_level);
// the last iteration's update (e += alpha p, ||r||^2), no V-cycle after it
void launch_cg_update_last(const MGHier &H, const CgVecs &v, int k, hipStream_t s);

// field.hip
struct FieldDev {
    int32_t nr, nz;
    double dr, dz;
    const double *ce64, *cn64;  // FP64 couplings (with eps0)
    const uint8_t *kind;        // 0 unknown, 1 cathode, 2 grounded
    double *phi, *phi0, *phi_l;
    double *phi0_prev;          // phi0 of the previous step (warm-start extrapolation)
    double *r64;                // FP64 residual
    float *e32, *q32, *p32[2];  // inner CG vectors (finest level)
    float *q32b, *r32b, *w32;   // second q and r buffers, w = A z (CG fused into the V-cycle)
    double *cg_acc;             // slotted dots of the fused CG (MAX_PCG iterations)
    MGHier mg;                  // r32 = mg.lv[0].b, z32 = mg.lv[0].xu
    const double *b_r, *b_z;    // static nodal B
    const double *vdep;         // node volumes for densities
    const int32_t *gate;        // when set and nonzero, the solve's kernels return at once
};

// ---- direct solve of the separable field equation (fastsolve.hip) -----------
// Buffers of the sine-transform solve: S (Mp x Mp, the orthonormal sine
// transform over the nz - 1 unknown rows, zero padded to a multiple of 32),
// the right-hand side b and its transform bh (Mp x Np, Np = nr padded), the
// radial and axial couplings of an interior row and the eigenvalues of
// tridiag(-1, 2, -1).
struct FastSolve {
    const double *S;
    double *b, *bh;
    const double *ce1, *cn1, *lam;
};
int fs_pad(int n);
// true when the unknowns are exactly i < nr, 0 < j < nz and the couplings
// are the same on every row (the cathode covers the z = 0 row)
bool fs_separable(int nr, int nz, const double *ce, const double *cn, const uint8_t *kind);
void fs_tables(int nr, int nz, const double *ce, const double *cn, double *S, double *ce1,
               double *cn1, double *lam);
// phi += K^-1 r on the unknown nodes, r = f.r64 the FP64 residual of phi
// (written by launch_residual64); also clears sc->res_slots for the residual
// check that follows
void launch_fast_solve(const FastSolve &F, const FieldDev &f, double *phi, DevScalars *sc,
                       hipStream_t s);

// ---- batched field update of an ensemble ------------------------------------

// Per-run descriptor in the run's workspace: the field state, the charge,
// the gather fields and the constants of the solve and the circuit; gates
// of f point at sc->solve_done.
struct RunSolve {
    FieldDev f;
    DevScalars *sc;
    const void *q0, *q1;        // node charge per species (state precision)
    void *node;                 // gather 4-vectors
    double rtol2;
    double v_fixed, v_ext, r_ext, dt, extra_dq, inv_2pi_eps0;
    int32_t circuit, scheme;
    CgVecs cg;                  // the run's CG vectors of the fused V-cycle
};

// Kernel argument of a batched launch: the runs and the first block of each.
struct BatchArgs {
    const RunSolve *run[MAX_BATCH];
    int32_t off[MAX_BATCH + 1];
    int32_t nruns;
    int32_t level, k, n_iter, op;
};

__device__ __forceinline__ int batch_run(const BatchArgs &a)
{
    int lo = 0, hi = a.nruns - 1;
    const int b = (int)blockIdx.x;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (a.off[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Host view of a batch: device descriptors and host copies of the shapes.
struct BatchPlan {
    int32_t nruns;
    const RunSolve *dev[MAX_BATCH];
    MGHier host[MAX_BATCH];
    int32_t prec;               // PIC_F32 or PIC_F64, common to the batch
};

void launch_mg_vcycle_b(const BatchPlan &P, int k, hipStream_t s);
void launch_cg_matvec_b(const BatchPlan &P, int k, hipStream_t s);
void launch_cg_update_b(const BatchPlan &P, int k, hipStream_t s);
// the fused forms (CG vector work in the finest level's V-cycle kernels) for
// batches whose every run has a finest level outside the coarse tail
bool batch_fused_cg(const BatchPlan &P);
void launch_mg_vcycle_cg_b(const BatchPlan &P, int k, hipStream_t s);
void launch_cg_update_last_b(const BatchPlan &P, int k, hipStream_t s);
// node-wise field operations of every run (op: BATCH_*), gated ones skip
// runs whose solve is done; BATCH_CAST_SCALE_CG also clears the slotted dots
// of n_iter fused CG iterations
enum : int32_t {
    BATCH_EXTRAPOLATE = 0, BATCH_SET_DIRICHLET = 1, BATCH_ZERO_IF_EMPTY = 2,
    BATCH_CAST_SCALE = 3, BATCH_UPDATE64 = 4, BATCH_FIELD_PREP = 5, BATCH_CAST_SCALE_CG = 6
};
void launch_nodes_b(const BatchPlan &P, int op, hipStream_t s, int n_iter = 0);
// per-run scalar operations (one block per run)
enum : int32_t {
    BATCH_ZERO_RES = 0, BATCH_ZERO_RES_GATED = 1, BATCH_SOLVE_INIT = 2, BATCH_SOLVE_GATE = 3,
    BATCH_ZERO_PCG_GATED = 4
};
void launch_scalars_b(const BatchPlan &P, int op, int n_iter, hipStream_t s);
void launch_residual64_b(const BatchPlan &P, int gated, hipStream_t s);
void launch_circuit_b(const BatchPlan &P, hipStream_t s);
// status of every run (residual norms, flags, counts, solve control) into
// host-mapped memory
struct RunStatus {
    double rr, bb, rr0;
    int32_t flags, pad;
    int64_t count[2];
    int32_t solve_done, solve_passes, solve_iters, solve_pad;
};
void launch_status_b(const BatchPlan &P, RunStatus *status_dev, hipStream_t s);

void launch_zero(void *p, int64_t bytes, hipStream_t s);
void launch_zero_gated(void *p, int64_t bytes, const int32_t *gate, hipStream_t s);
// FP64 residual and its norms (zero: clear the accumulators first; false when
// an earlier kernel of the sequence has)
template <typename T>
void launch_residual64(const FieldDev &f, const double *phi, const T *q0, const T *q1,
                       DevScalars *sc, hipStream_t s, bool zero = true);
// out = K phi on unknown nodes, 0 on Dirichlet nodes (FP64)
void launch_apply_k64(const FieldDev &f, const double *phi, double *out, hipStream_t s);
// r32 = r64 / ||r64|| (norm read on the device), e32 = 0, and nzero doubles
// at zero cleared
void launch_cast_scale(const FieldDev &f, DevScalars *sc, hipStream_t s, double *zero = nullptr,
                       int64_t nzero = 0);
// phi += e32 ||r64|| / (2 pi eps0) on unknown nodes; zero_res also clears
// the residual accumulators for the residual that follows; with cg_iters > 0
// it also sums the fused CG's slotted ||r||^2 of each iteration into
// sc->pcg_rr
void launch_update64(const FieldDev &f, double *phi, DevScalars *sc, double inv_2pi_eps0,
                     hipStream_t s, bool zero_res = false, int cg_iters = 0);
// extrapolation of phi0 (when asked), Dirichlet values, cleared residual
// accumulators: the start of a solve in one launch
void launch_solve_prep(const FieldDev &f, double *phi, bool extrapolate, double v_cathode,
                       DevScalars *sc, hipStream_t s);
template <typename T>
void launch_circuit(const FieldDev &f, const T *q0, const T *q1, DevScalars *sc, int circuit,
                    double v_fixed, double v_ext, double r_ext, double dt, double extra_dq,
                    hipStream_t s, double check_rtol2 = 0.0);
template <typename T>
void launch_field_prep(const FieldDev &f, typename Vec4<T>::type *node, DevScalars *sc,
                       int scheme, int use_phi, hipStream_t s);
void launch_set_dirichlet(const FieldDev &f, double *phi, double v_cathode, hipStream_t s);
template <typename T>
void launch_diag_grid(const FieldDev &f, const T *q0, const T *q1, double q_e, double q_i,
                      double *partials, int nblocks, hipStream_t s);
void launch_count_live(const int32_t *key, const DevScalars *sc, int species,
                       unsigned long long *out, hipStream_t s);
void launch_zero_unknowns(const FieldDev &f, double *phi, hipStream_t s);
// phi0 <- 2 phi0 - phi0_prev, phi0_prev <- phi0 (unknown nodes); copy when first
void launch_extrapolate(const FieldDev &f, int first, hipStream_t s);

// host_tables.cpp (FP64 host arithmetic, built without FMA contraction)
double host_nu_tables(const pic_config &c, double *nu, unsigned long long *t_null);
unsigned long long host_see_threshold(const pic_config &c, int species);
void host_couplings(int nr, int nz, double lr, double lz, double scale, double *ce, double *cn);
int host_node_kind(int nr, int nz, double lr, double cathode_rmax, int i, int j);
int host_dense_inverse(int n, double *a);   // in place, returns 0 on success
double eps0();
void host_node_volumes(int nr, int nz, double lr, double lz, double *v);

}  // namespace pic
