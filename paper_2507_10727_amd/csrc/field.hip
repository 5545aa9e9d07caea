// Field kernels of libpic.so: FP64 residual and refinement of the R-Z
// charge-form operator, the cathode circuit, the gather-field packing and
// grid diagnostics (the FP32 multigrid/CG inner solve is in mg.hip).
//
// Operator (reading of Section 3's "Gauss' law is obeyed along this axis"):
//   (K phi)_n = sum over the faces f of node n of c_f (phi_n - phi_nb),
// c_f = eps0 A_f / h_f of the clipped control volume; Dirichlet nodes are the
// anode row, the outer column and the cathode part of z = 0.  The FP32
// inner solve (mg.hip) works on K / (2 pi eps0) for the correction equation
// K_uu e = r of the FP64 refinement, with zero correction on Dirichlet
// nodes.
#include <cstring>

#include <algorithm>

#include "common.h"

namespace pic {

namespace {

constexpr int FB = 256;
// Kernels that end in a block sum added atomically to one FP64 scalar run
// few large blocks: atomics on one address are serialized (about 15 ns each),
// so 1024 blocks of 256 threads spent ~15 us in them where 256 blocks of
// 1024 threads spend a quarter of that.
constexpr int RB = 1024;
inline int res_blocks(int64_t n)
{
    int64_t b = (n + RB - 1) / RB;
    return (int)std::max<int64_t>(1, std::min<int64_t>(b, 256));
}

inline int blocks_for(int64_t n, int cap = 4096)
{
    int64_t b = (n + FB - 1) / FB;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (int)b;
}

__device__ __forceinline__ double block_sum(double v, double *buf)
{
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) buf[wid] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += buf[w];
    __syncthreads();
    return t;   // valid in thread 0
}

__global__ void k_zero(uint32_t *p, int64_t words, const int32_t *gate)
{
    if (gate && *gate) return;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < words;
         k += (int64_t)gridDim.x * blockDim.x)
        p[k] = 0u;
}

template <typename T>
__device__ __forceinline__ double load_q(const T *q0, const T *q1, int64_t n)
{
    double v = (double)q0[n];
    if (q1) v += (double)q1[n];
    return v;
}

// r = q - K phi on unknown rows (0 elsewhere); accumulates ||r||^2 and
// ||b||^2 with b = q + couplings to Dirichlet neighbours (their phi values).
template <typename T>
__device__ __forceinline__ void residual64_body(int32_t nr, int32_t nz, const double *ce,
                                                   const double *cn, const uint8_t *kind,
                                                   const double *phi, const T *q0, const T *q1,
                                                   double *r64, DevScalars *sc,
                                                   const int32_t *gate, int blk, int nblk,
                                                   bool slotted = false)
{
    if (gate && *gate) return;
    __shared__ double buf[RB / 64];
    const int ld = nr + 1;
    const int64_t nn = (int64_t)ld * (nz + 1);
    double rr = 0.0, bb = 0.0;
    for (int64_t n = (int64_t)blk * RB + threadIdx.x; n < nn; n += (int64_t)nblk * RB) {
        if (kind[n] != 0) { r64[n] = 0.0; continue; }
        int i, j;
        node_ij(n, ld, i, j);
        const double p = phi[n];
        double flux = 0.0, dir = 0.0;
        if (i < nr) { const double c = ce[n]; flux += c * (p - phi[n + 1]); if (kind[n + 1]) dir += c * phi[n + 1]; }
        if (i > 0) { const double c = ce[n - 1]; flux += c * (p - phi[n - 1]); if (kind[n - 1]) dir += c * phi[n - 1]; }
        if (j < nz) { const double c = cn[n]; flux += c * (p - phi[n + ld]); if (kind[n + ld]) dir += c * phi[n + ld]; }
        if (j > 0) { const double c = cn[n - ld]; flux += c * (p - phi[n - ld]); if (kind[n - ld]) dir += c * phi[n - ld]; }
        const double q = load_q(q0, q1, n);
        const double r = q - flux;
        r64[n] = r;
        rr += r * r;
        bb += (q + dir) * (q + dir);
    }
    const double a = block_sum(rr, buf);
    const double b = block_sum(bb, buf);
    if (threadIdx.x == 0) {
        if (slotted) {
            // (blocks finishing together would serialize on one address)
            const int sl = (blk & (ACC_SLOTS - 1)) * ACC_STRIDE;
            if (a != 0.0) atomic_add_dev(&sc->res_slots[sl], a);
            if (b != 0.0) atomic_add_dev(&sc->res_slots[ACC_SLOTS * ACC_STRIDE + sl], b);
        } else {
            if (a != 0.0) atomic_add_dev(&sc->res_rr, a);
            if (b != 0.0) atomic_add_dev(&sc->res_bb, b);
        }
    }
}

template <typename T>
__global__ void __launch_bounds__(RB) k_residual64(int32_t nr, int32_t nz, const double *ce,
                                                   const double *cn, const uint8_t *kind,
                                                   const double *phi, const T *q0, const T *q1,
                                                   double *r64, DevScalars *sc,
                                                   const int32_t *gate)
{
    residual64_body<T>(nr, nz, ce, cn, kind, phi, q0, q1, r64, sc, gate, blockIdx.x, gridDim.x,
                       true);
}

// out = K phi on unknown nodes (charge form, C), 0 on Dirichlet nodes
__global__ void __launch_bounds__(FB) k_apply_k64(int32_t nr, int32_t nz, const double *ce,
                                                  const double *cn, const uint8_t *kind,
                                                  const double *phi, double *out)
{
    const int ld = nr + 1;
    const int64_t nn = (int64_t)ld * (nz + 1);
    for (int64_t n = (int64_t)blockIdx.x * FB + threadIdx.x; n < nn; n += (int64_t)gridDim.x * FB) {
        if (kind[n] != 0) { out[n] = 0.0; continue; }
        int i, j;
        node_ij(n, ld, i, j);
        const double p = phi[n];
        double flux = 0.0;
        if (i < nr) flux += ce[n] * (p - phi[n + 1]);
        if (i > 0) flux += ce[n - 1] * (p - phi[n - 1]);
        if (j < nz) flux += cn[n] * (p - phi[n + ld]);
        if (j > 0) flux += cn[n - ld] * (p - phi[n - ld]);
        out[n] = flux;
    }
}

// also zeroes nzero doubles at zero (the pass's CG accumulators), which
// nothing in this kernel reads
__device__ __forceinline__ void cast_scale_body(int64_t nn, const double *r64, DevScalars *sc, float *r32, float *e32,
                             const int32_t *gate, int blk, int nblk, double *zero = nullptr,
                             int64_t nzero = 0, bool slotted = false)
{
    if (gate && *gate) return;
    double rr;
    if (slotted) {
        // the residual's slots, lane l reading slot l mod ACC_SLOTS, summed
        // by a butterfly that leaves the same sum in every lane
        rr = sc->res_slots[(threadIdx.x & (ACC_SLOTS - 1)) * ACC_STRIDE];
        for (int o = ACC_SLOTS / 2; o > 0; o >>= 1) rr += __shfl_xor(rr, o, ACC_SLOTS);
    } else {
        rr = sc->res_rr;
    }
    const double scale = (rr > 0.0) ? 1.0 / sqrt(rr) : 0.0;
    if (blk == 0 && threadIdx.x == 0) sc->res_rr0 = rr;
    for (int64_t k = (int64_t)blk * FB + threadIdx.x; k < nzero; k += (int64_t)nblk * FB)
        zero[k] = 0.0;
    for (int64_t n = (int64_t)blk * FB + threadIdx.x; n < nn; n += (int64_t)nblk * FB) {
        r32[n] = (float)(r64[n] * scale);
        e32[n] = 0.0f;
    }
}

__global__ void k_cast_scale(int64_t nn, const double *r64, DevScalars *sc, float *r32, float *e32,
                             const int32_t *gate, double *zero, int64_t nzero)
{
    cast_scale_body(nn, r64, sc, r32, e32, gate, blockIdx.x, gridDim.x, zero, nzero, true);
}

// with zero_res, also zeroes the residual accumulators (res_rr, res_bb) for
// the residual that follows; this kernel reads only res_rr0
__device__ __forceinline__ void update64_body(int64_t nn, const uint8_t *kind, double *phi, const float *e32,
                           const DevScalars *sc, double inv_2pi_eps0, const int32_t *gate, int blk, int nblk,
                           double *zero_res = nullptr, const double *cg_acc = nullptr,
                           double *rr_out = nullptr, int cg_iters = 0)
{
    if (gate && *gate) return;
    const double scale = sqrt(sc->res_rr0) * inv_2pi_eps0;
    if (zero_res && blk == 0)
        for (int k = threadIdx.x; k < RES_SLOT_WORDS; k += FB) zero_res[k] = 0.0;
    if (blk == 0)
        for (int k = threadIdx.x; k < cg_iters; k += FB) {
            double a = 0.0;
            for (int sl = 0; sl < CG_SLOTS; ++sl) a += cg_acc[cg_acc_at(k, 3, sl)];
            rr_out[k] = a;
        }
    for (int64_t n = (int64_t)blk * FB + threadIdx.x; n < nn; n += (int64_t)nblk * FB)
        if (kind[n] == 0) phi[n] += (double)e32[n] * scale;
}

__global__ void k_update64(int64_t nn, const uint8_t *kind, double *phi, const float *e32,
                           const DevScalars *sc, double inv_2pi_eps0, const int32_t *gate,
                           double *zero_res, const double *cg_acc, double *rr_out, int cg_iters)
{
    update64_body(nn, kind, phi, e32, sc, inv_2pi_eps0, gate, blockIdx.x, gridDim.x, zero_res,
                  cg_acc, rr_out, cg_iters);
}

// ---- circuit: induced cathode charge of phi0 and the cathode voltage update
template <typename T>
__device__ __forceinline__ void circuit_body(int32_t nr, const double *ce, const double *cn, const uint8_t *kind,
                          const double *phi0, const T *q0, const T *q1, DevScalars *sc,
                          int circuit, double v_fixed, double v_ext, double r_ext, double dt,
                          double extra_dq, int blk, int nblk)
{
    __shared__ double buf[1024 / 64];
    const int ld = nr + 1;
    double acc = 0.0;
    for (int i = threadIdx.x; i <= nr; i += blockDim.x) {
        if (kind[i] != 1) continue;
        const int64_t n = i;
        const double p = phi0[n];
        double flux = 0.0;
        if (i < nr) flux += ce[n] * (p - phi0[n + 1]);
        if (i > 0) flux += ce[n - 1] * (p - phi0[n - 1]);
        flux += cn[n] * (p - phi0[n + ld]);
        acc += flux - load_q(q0, q1, n);
    }
    const double qc0 = block_sum(acc, buf);
    if (threadIdx.x == 0) {
        const double dq = sc->dq_conv + extra_dq;
        sc->dq_conv = dq;
        double v;
        if (circuit == PIC_RESISTOR)
            v = (sc->qc + dq + dt * v_ext / r_ext - qc0) / (sc->cap_c + dt / r_ext);
        else
            v = v_fixed;
        sc->qc0 = qc0;
        sc->vc = v;
        sc->qc = qc0 + sc->cap_c * v;
    }
}

template <typename T>
__global__ void k_circuit(int32_t nr, const double *ce, const double *cn, const uint8_t *kind,
                          const double *phi0, const T *q0, const T *q1, DevScalars *sc,
                          int circuit, double v_fixed, double v_ext, double r_ext, double dt,
                          double extra_dq, double check_rtol2)
{
    // the preceding direct solve's check (check_rtol2 > 0): FLAG_NOCONV when
    // its residual (slotted norms) exceeds the tolerance
    if (check_rtol2 > 0.0 && blockIdx.x == 0 && threadIdx.x == 0) {
        double rr = 0.0, bb = 0.0;
        for (int k = 0; k < ACC_SLOTS; ++k) {
            rr += sc->res_slots[k * ACC_STRIDE];
            bb += sc->res_slots[(ACC_SLOTS + k) * ACC_STRIDE];
        }
        if (!(rr <= check_rtol2 * bb)) atomicOr(&sc->flags, FLAG_NOCONV);
    }
    circuit_body<T>(nr, ce, cn, kind, phi0, q0, q1, sc, circuit, v_fixed, v_ext, r_ext, dt, extra_dq, blockIdx.x, gridDim.x);
}

// ---- gather fields: phi = phi0 + V_c phi_L and the node 4-vectors
template <typename T>
__device__ __forceinline__ void field_prep_body(int32_t nr, int32_t nz, double dr, double dz, double *phi,
                             const double *phi0, const double *phil, const double *br,
                             const double *bz, typename Vec4<T>::type *node, const DevScalars *sc,
                             int scheme, int use_phi, int blk, int nblk)
{
    const int ld = nr + 1;
    const int64_t nn = (int64_t)ld * (nz + 1);
    const double vc = sc->vc;
    for (int64_t n = (int64_t)blk * FB + threadIdx.x; n < nn; n += (int64_t)nblk * FB) {
        int i, j;
        node_ij(n, ld, i, j);
#define PHI(m) (use_phi ? phi[(m)] : (phi0[(m)] + vc * phil[(m)]))
        const double p = PHI(n);
        double ex, ey;
        if (scheme == PIC_EC) {
            ex = (i < nr) ? -(PHI(n + 1) - p) / dr : 0.0;
            ey = (j < nz) ? -(PHI(n + ld) - p) / dz : 0.0;
        } else {
            if (i == 0) ex = 0.0;
            else if (i == nr) ex = -(p - PHI(n - 1)) / dr;
            else ex = -(PHI(n + 1) - PHI(n - 1)) / (2.0 * dr);
            if (j == 0) ey = -(PHI(n + ld) - p) / dz;
            else if (j == nz) ey = -(p - PHI(n - ld)) / dz;
            else ey = -(PHI(n + ld) - PHI(n - ld)) / (2.0 * dz);
        }
#undef PHI
        if (!use_phi) phi[n] = p;
        typename Vec4<T>::type v;
        v.x = (T)ex;
        v.y = (T)ey;
        v.z = (T)br[n];
        v.w = (T)bz[n];
        node[n] = v;
    }
}

template <typename T>
__global__ void k_field_prep(int32_t nr, int32_t nz, double dr, double dz, double *phi,
                             const double *phi0, const double *phil, const double *br,
                             const double *bz, typename Vec4<T>::type *node, const DevScalars *sc,
                             int scheme, int use_phi)
{
    field_prep_body<T>(nr, nz, dr, dz, phi, phi0, phil, br, bz, node, sc, scheme, use_phi, blockIdx.x, gridDim.x);
}

__global__ void k_zero_unknowns(int64_t nn, const uint8_t *kind, double *phi)
{
    for (int64_t n = (int64_t)blockIdx.x * FB + threadIdx.x; n < nn; n += (int64_t)gridDim.x * FB)
        if (kind[n] == 0) phi[n] = 0.0;
}

__device__ __forceinline__ void extrapolate_body(int64_t nn, const uint8_t *kind, double *phi0, double *prev,
                              int first, int blk, int nblk)
{
    for (int64_t n = (int64_t)blk * FB + threadIdx.x; n < nn; n += (int64_t)nblk * FB) {
        const double t = phi0[n];
        if (!first && kind[n] == 0) phi0[n] = 2.0 * t - prev[n];
        prev[n] = t;
    }
}

__global__ void k_extrapolate(int64_t nn, const uint8_t *kind, double *phi0, double *prev,
                              int first)
{
    extrapolate_body(nn, kind, phi0, prev, first, blockIdx.x, gridDim.x);
}

__device__ __forceinline__ void set_dirichlet_body(int64_t nn, const uint8_t *kind, double *phi, double vcat, int blk, int nblk)
{
    for (int64_t n = (int64_t)blk * FB + threadIdx.x; n < nn; n += (int64_t)nblk * FB) {
        if (kind[n] == 1) phi[n] = vcat;
        else if (kind[n] == 2) phi[n] = 0.0;
    }
}

__global__ void k_set_dirichlet(int64_t nn, const uint8_t *kind, double *phi, double vcat)
{
    set_dirichlet_body(nn, kind, phi, vcat, blockIdx.x, gridDim.x);
}

// Start of a solve in one launch: the warm-start extrapolation of the
// unknowns (when prev is given), the Dirichlet values, and zeroed residual
// accumulators for the residual that follows.
__global__ void k_solve_prep(int64_t nn, const uint8_t *kind, double *phi, double *prev,
                             double vcat, double *zero_res)
{
    if (blockIdx.x == 0)
        for (int k = threadIdx.x; k < RES_SLOT_WORDS; k += FB) zero_res[k] = 0.0;
    for (int64_t n = (int64_t)blockIdx.x * FB + threadIdx.x; n < nn; n += (int64_t)gridDim.x * FB) {
        const uint8_t k = kind[n];
        if (prev) {
            const double t = phi[n];
            if (k == 0) phi[n] = 2.0 * t - prev[n];
            prev[n] = t;
        }
        if (k == 1) phi[n] = vcat;
        else if (k == 2) phi[n] = 0.0;
    }
}

// Per-block partial diagnostics: sum Q_e, sum Q_i, max n_e, max n_i, max phi,
// field energy 1/2 sum_faces c (dphi)^2.
template <typename T>
__global__ void __launch_bounds__(FB) k_diag_grid(int32_t nr, int32_t nz, const double *ce,
                                                  const double *cn, const double *phi,
                                                  const double *vdep, const T *q0, const T *q1,
                                                  double qe, double qi, double *partials)
{
    __shared__ double buf[6][FB];
    const int ld = nr + 1;
    const int64_t nn = (int64_t)ld * (nz + 1);
    double s0 = 0, s1 = 0, m0 = -1e300, m1 = -1e300, mp = -1e300, w = 0;
    for (int64_t n = (int64_t)blockIdx.x * FB + threadIdx.x; n < nn; n += (int64_t)gridDim.x * FB) {
        int i, j;
        node_ij(n, ld, i, j);
        const double a = (double)q0[n], b = (double)q1[n];
        s0 += a;
        s1 += b;
        m0 = fmax(m0, a / (qe * vdep[n]));
        m1 = fmax(m1, b / (qi * vdep[n]));
        mp = fmax(mp, phi[n]);
        if (i < nr) { const double d = phi[n] - phi[n + 1]; w += 0.5 * ce[n] * d * d; }
        if (j < nz) { const double d = phi[n] - phi[n + ld]; w += 0.5 * cn[n] * d * d; }
    }
    const int t = threadIdx.x;
    buf[0][t] = s0; buf[1][t] = s1; buf[2][t] = m0; buf[3][t] = m1; buf[4][t] = mp; buf[5][t] = w;
    __syncthreads();
    for (int o = FB / 2; o > 0; o >>= 1) {
        if (t < o) {
            buf[0][t] += buf[0][t + o];
            buf[1][t] += buf[1][t + o];
            buf[2][t] = fmax(buf[2][t], buf[2][t + o]);
            buf[3][t] = fmax(buf[3][t], buf[3][t + o]);
            buf[4][t] = fmax(buf[4][t], buf[4][t + o]);
            buf[5][t] += buf[5][t + o];
        }
        __syncthreads();
    }
    if (t < 6) partials[blockIdx.x * 6 + t] = buf[t][0];
}

__global__ void k_count_live(const int32_t *key, const DevScalars *sc, int species,
                             unsigned long long *out)
{
    const int64_t n = sc->count[species];
    unsigned long long c = 0;
    for (int64_t p = (int64_t)blockIdx.x * FB + threadIdx.x; p < n; p += (int64_t)gridDim.x * FB)
        c += (key[p] >= 0) ? 1ull : 0ull;
    c = wave_sum_u64(c);
    if ((threadIdx.x & 63) == 0 && c) atomicAdd(out, c);
}

__device__ __forceinline__ void zero_unknowns_if_empty_body(int64_t nn, const uint8_t *kind, double *phi,
                                         const DevScalars *sc, int blk, int nblk)
{
    if (sc->res_bb != 0.0) return;
    for (int64_t n = (int64_t)blk * FB + threadIdx.x; n < nn; n += (int64_t)nblk * FB)
        if (kind[n] == 0) phi[n] = 0.0;
}

// ---- batched forms over the runs of an ensemble ------------------------------
template <typename T>
__global__ void __launch_bounds__(FB) k_nodes_b(BatchArgs a)
{
    const int r = batch_run(a);
    const RunSolve &R = *a.run[r];
    const FieldDev &f = R.f;
    const int blk = (int)blockIdx.x - a.off[r], nblk = a.off[r + 1] - a.off[r];
    const int64_t nn = (int64_t)(f.nr + 1) * (f.nz + 1);
    switch (a.op) {
        case BATCH_EXTRAPOLATE:
            extrapolate_body(nn, f.kind, f.phi0, f.phi0_prev, 0, blk, nblk);
            break;
        case BATCH_SET_DIRICHLET: set_dirichlet_body(nn, f.kind, f.phi0, 0.0, blk, nblk); break;
        case BATCH_ZERO_IF_EMPTY:
            zero_unknowns_if_empty_body(nn, f.kind, f.phi0, R.sc, blk, nblk);
            break;
        case BATCH_CAST_SCALE:
            cast_scale_body(nn, f.r64, R.sc, f.mg.lv[0].b, f.e32, f.gate, blk, nblk);
            break;
        case BATCH_UPDATE64:
            update64_body(nn, f.kind, f.phi0, f.e32, R.sc, R.inv_2pi_eps0, f.gate, blk, nblk);
            break;
        case BATCH_CAST_SCALE_CG:
            cast_scale_body(nn, f.r64, R.sc, f.mg.lv[0].b, f.e32, f.gate, blk, nblk, R.cg.acc,
                            (int64_t)a.n_iter * CG_ACC_PER_ITER);
            break;
        default:
            // runs whose solve has converged and whose step is not finished
            if (!R.sc->solve_done || R.sc->post_done) return;
            field_prep_body<T>(f.nr, f.nz, f.dr, f.dz, f.phi, f.phi0, f.phi_l, f.b_r, f.b_z,
                               (typename Vec4<T>::type *)R.node, R.sc, R.scheme, 0, blk, nblk);
            break;
    }
}

__global__ void k_scalars_b(BatchArgs a)
{
    const RunSolve &R = *a.run[blockIdx.x];
    DevScalars *sc = R.sc;
    const bool done = sc->solve_done != 0;
    switch (a.op) {
        case BATCH_ZERO_RES:
        case BATCH_ZERO_RES_GATED:
            if (threadIdx.x == 0 && !(a.op == BATCH_ZERO_RES_GATED && done)) {
                sc->res_rr = 0.0;
                sc->res_bb = 0.0;
            }
            break;
        case BATCH_SOLVE_INIT:
            if (threadIdx.x == 0) {
                const double rr = sc->res_rr, bb = sc->res_bb;
                sc->solve_done = (bb == 0.0 || rr <= R.rtol2 * bb) ? 1 : 0;
                sc->post_done = 0;
                sc->solve_passes = 0;
                sc->solve_iters = 0;
            }
            break;
        case BATCH_SOLVE_GATE:
            if (threadIdx.x == 0 && !done) {
                sc->solve_passes += 1;
                sc->solve_iters += a.n_iter;
                const double rr = sc->res_rr, bb = sc->res_bb;
                sc->solve_done = (bb == 0.0 || rr <= R.rtol2 * bb) ? 1 : 0;
            }
            break;
        default:
            if (!done)
                for (int t = threadIdx.x; t < 5 * (MAX_PCG + 2); t += blockDim.x) sc->pcg_rz[t] = 0.0;
            break;
    }
}

template <typename T>
__global__ void __launch_bounds__(RB) k_residual64_b(BatchArgs a)
{
    const int r = batch_run(a);
    const RunSolve &R = *a.run[r];
    const FieldDev &f = R.f;
    residual64_body<T>(f.nr, f.nz, f.ce64, f.cn64, f.kind, f.phi0, (const T *)R.q0,
                       (const T *)R.q1, f.r64, R.sc, a.op ? f.gate : nullptr,
                       (int)blockIdx.x - a.off[r], a.off[r + 1] - a.off[r]);
}

template <typename T>
__global__ void k_circuit_b(BatchArgs a)
{
    const RunSolve &R = *a.run[blockIdx.x];
    const FieldDev &f = R.f;
    if (!R.sc->solve_done || R.sc->post_done) return;
    circuit_body<T>(f.nr, f.ce64, f.cn64, f.kind, f.phi0, (const T *)R.q0, (const T *)R.q1, R.sc,
                    R.circuit, R.v_fixed, R.v_ext, R.r_ext, R.dt, R.extra_dq, 0, 1);
}

__global__ void k_status_b(BatchArgs a, RunStatus *out)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= a.nruns) return;
    DevScalars *sc = a.run[r]->sc;
    if (sc->solve_done) sc->post_done = 1;
    RunStatus s;
    s.rr = sc->res_rr;
    s.bb = sc->res_bb;
    s.rr0 = sc->res_rr0;
    s.flags = sc->flags;
    s.pad = 0;
    s.count[0] = sc->count[0];
    s.count[1] = sc->count[1];
    s.solve_done = sc->solve_done;
    s.solve_passes = sc->solve_passes;
    s.solve_iters = sc->solve_iters;
    s.solve_pad = 0;
    out[r] = s;
}

BatchArgs node_args(const BatchPlan &P, int op)
{
    BatchArgs a;
    memset(&a, 0, sizeof(a));
    a.nruns = P.nruns;
    a.op = op;
    for (int r = 0; r < P.nruns; ++r) {
        a.run[r] = P.dev[r];
        const int64_t nn = (int64_t)(P.host[r].lv[0].nr + 1) * (P.host[r].lv[0].nz + 1);
        a.off[r + 1] = a.off[r] + blocks_for((nn + 1) / 2, 1024);
    }
    return a;
}

BatchArgs run_args(const BatchPlan &P, int op)
{
    BatchArgs a;
    memset(&a, 0, sizeof(a));
    a.nruns = P.nruns;
    a.op = op;
    for (int r = 0; r < P.nruns; ++r) {
        a.run[r] = P.dev[r];
        a.off[r + 1] = r + 1;
    }
    return a;
}

}  // namespace

void launch_zero(void *p, int64_t bytes, hipStream_t s)
{
    const int64_t words = (bytes + 3) / 4;
    hipLaunchKernelGGL(k_zero, dim3(blocks_for(words, 2048)), dim3(FB), 0, s, (uint32_t *)p, words,
                       (const int32_t *)nullptr);
}

void launch_zero_gated(void *p, int64_t bytes, const int32_t *gate, hipStream_t s)
{
    const int64_t words = (bytes + 3) / 4;
    hipLaunchKernelGGL(k_zero, dim3(blocks_for(words, 2048)), dim3(FB), 0, s, (uint32_t *)p, words,
                       gate);
}


template <typename T>
void launch_residual64(const FieldDev &f, const double *phi, const T *q0, const T *q1,
                       DevScalars *sc, hipStream_t s, bool zero)
{
    const int64_t nn = (int64_t)(f.nr + 1) * (f.nz + 1);
    if (zero) launch_zero_gated(sc->res_slots, RES_SLOT_WORDS * sizeof(double), f.gate, s);
    hipLaunchKernelGGL((k_residual64<T>), dim3(res_blocks(nn)), dim3(RB), 0, s, f.nr,
                       f.nz, f.ce64, f.cn64, f.kind, phi, q0, q1, f.r64, sc, f.gate);
}

void launch_apply_k64(const FieldDev &f, const double *phi, double *out, hipStream_t s)
{
    const int64_t nn = (int64_t)(f.nr + 1) * (f.nz + 1);
    hipLaunchKernelGGL(k_apply_k64, dim3(blocks_for(nn)), dim3(FB), 0, s, f.nr, f.nz, f.ce64,
                       f.cn64, f.kind, phi, out);
}

void launch_cast_scale(const FieldDev &f, DevScalars *sc, hipStream_t s, double *zero,
                       int64_t nzero)
{
    const int64_t nn = (int64_t)(f.nr + 1) * (f.nz + 1);
    hipLaunchKernelGGL(k_cast_scale, dim3(blocks_for(nn)), dim3(FB), 0, s, nn, f.r64, sc,
                       f.mg.lv[0].b, f.e32, f.gate, zero, nzero);
}

void launch_update64(const FieldDev &f, double *phi, DevScalars *sc, double inv_2pi_eps0,
                     hipStream_t s, bool zero_res, int cg_iters)
{
    const int64_t nn = (int64_t)(f.nr + 1) * (f.nz + 1);
    hipLaunchKernelGGL(k_update64, dim3(blocks_for(nn)), dim3(FB), 0, s, nn, f.kind, phi, f.e32,
                       sc, inv_2pi_eps0, f.gate, zero_res ? sc->res_slots : nullptr, f.cg_acc,
                       sc->pcg_rr, cg_iters);
}

void launch_solve_prep(const FieldDev &f, double *phi, bool extrapolate, double v_cathode,
                       DevScalars *sc, hipStream_t s)
{
    const int64_t nn = (int64_t)(f.nr + 1) * (f.nz + 1);
    hipLaunchKernelGGL(k_solve_prep, dim3(blocks_for(nn)), dim3(FB), 0, s, nn, f.kind, phi,
                       extrapolate ? f.phi0_prev : nullptr, v_cathode, sc->res_slots);
}

template <typename T>
void launch_circuit(const FieldDev &f, const T *q0, const T *q1, DevScalars *sc, int circuit,
                    double v_fixed, double v_ext, double r_ext, double dt, double extra_dq,
                    hipStream_t s, double check_rtol2)
{
    hipLaunchKernelGGL((k_circuit<T>), dim3(1), dim3(1024), 0, s, f.nr, f.ce64, f.cn64, f.kind,
                       f.phi0, q0, q1, sc, circuit, v_fixed, v_ext, r_ext, dt, extra_dq,
                       check_rtol2);
}

template <typename T>
void launch_field_prep(const FieldDev &f, typename Vec4<T>::type *node, DevScalars *sc,
                       int scheme, int use_phi, hipStream_t s)
{
    const int64_t nn = (int64_t)(f.nr + 1) * (f.nz + 1);
    hipLaunchKernelGGL((k_field_prep<T>), dim3(blocks_for(nn)), dim3(FB), 0, s, f.nr, f.nz, f.dr,
                       f.dz, f.phi, f.phi0, f.phi_l, f.b_r, f.b_z, node, sc, scheme, use_phi);
}

void launch_extrapolate(const FieldDev &f, int first, hipStream_t s)
{
    const int64_t nn = (int64_t)(f.nr + 1) * (f.nz + 1);
    hipLaunchKernelGGL(k_extrapolate, dim3(blocks_for(nn)), dim3(FB), 0, s, nn, f.kind, f.phi0,
                       f.phi0_prev, first);
}

void launch_set_dirichlet(const FieldDev &f, double *phi, double v_cathode, hipStream_t s)
{
    const int64_t nn = (int64_t)(f.nr + 1) * (f.nz + 1);
    hipLaunchKernelGGL(k_set_dirichlet, dim3(blocks_for(nn)), dim3(FB), 0, s, nn, f.kind, phi,
                       v_cathode);
}

void launch_zero_unknowns(const FieldDev &f, double *phi, hipStream_t s)
{
    const int64_t nn = (int64_t)(f.nr + 1) * (f.nz + 1);
    hipLaunchKernelGGL(k_zero_unknowns, dim3(blocks_for(nn)), dim3(FB), 0, s, nn, f.kind, phi);
}

template <typename T>
void launch_diag_grid(const FieldDev &f, const T *q0, const T *q1, double q_e, double q_i,
                      double *partials, int nblocks, hipStream_t s)
{
    hipLaunchKernelGGL((k_diag_grid<T>), dim3(nblocks), dim3(FB), 0, s, f.nr, f.nz, f.ce64, f.cn64,
                       f.phi, f.vdep, q0, q1, q_e, q_i, partials);
}

void launch_count_live(const int32_t *key, const DevScalars *sc, int species,
                       unsigned long long *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_count_live, dim3(1024), dim3(FB), 0, s, key, sc, species, out);
}

template void launch_residual64<float>(const FieldDev &, const double *, const float *,
                                       const float *, DevScalars *, hipStream_t, bool);
template void launch_residual64<double>(const FieldDev &, const double *, const double *,
                                        const double *, DevScalars *, hipStream_t, bool);
template void launch_circuit<float>(const FieldDev &, const float *, const float *, DevScalars *,
                                    int, double, double, double, double, double, hipStream_t,
                                    double);
template void launch_circuit<double>(const FieldDev &, const double *, const double *,
                                     DevScalars *, int, double, double, double, double, double,
                                     hipStream_t, double);
void launch_nodes_b(const BatchPlan &P, int op, hipStream_t s, int n_iter)
{
    BatchArgs a = node_args(P, op);
    a.n_iter = n_iter;
    if (P.prec == PIC_F64)
        hipLaunchKernelGGL(k_nodes_b<double>, dim3(a.off[P.nruns]), dim3(FB), 0, s, a);
    else
        hipLaunchKernelGGL(k_nodes_b<float>, dim3(a.off[P.nruns]), dim3(FB), 0, s, a);
}

void launch_scalars_b(const BatchPlan &P, int op, int n_iter, hipStream_t s)
{
    BatchArgs a = run_args(P, op);
    a.n_iter = n_iter;
    hipLaunchKernelGGL(k_scalars_b, dim3(P.nruns), dim3(256), 0, s, a);
}

void launch_residual64_b(const BatchPlan &P, int gated, hipStream_t s)
{
    BatchArgs a = node_args(P, gated);
    for (int r = 0; r < P.nruns; ++r)
        a.off[r + 1] = a.off[r] + res_blocks((int64_t)(P.host[r].lv[0].nr + 1) * (P.host[r].lv[0].nz + 1));
    if (P.prec == PIC_F64)
        hipLaunchKernelGGL(k_residual64_b<double>, dim3(a.off[P.nruns]), dim3(RB), 0, s, a);
    else
        hipLaunchKernelGGL(k_residual64_b<float>, dim3(a.off[P.nruns]), dim3(RB), 0, s, a);
}

void launch_circuit_b(const BatchPlan &P, hipStream_t s)
{
    const BatchArgs a = run_args(P, 0);
    if (P.prec == PIC_F64)
        hipLaunchKernelGGL(k_circuit_b<double>, dim3(P.nruns), dim3(1024), 0, s, a);
    else
        hipLaunchKernelGGL(k_circuit_b<float>, dim3(P.nruns), dim3(1024), 0, s, a);
}

void launch_status_b(const BatchPlan &P, RunStatus *status_dev, hipStream_t s)
{
    const BatchArgs a = run_args(P, 0);
    hipLaunchKernelGGL(k_status_b, dim3((P.nruns + 63) / 64), dim3(64), 0, s, a, status_dev);
}

template void launch_field_prep<float>(const FieldDev &, float4 *, DevScalars *, int, int,
                                       hipStream_t);
template void launch_field_prep<double>(const FieldDev &, double4 *, DevScalars *, int, int,
                                        hipStream_t);
template void launch_diag_grid<float>(const FieldDev &, const float *, const float *, double,
                                      double, double *, int, hipStream_t);
template void launch_diag_grid<double>(const FieldDev &, const double *, const double *, double,
                                       double, double *, int, hipStream_t);

}  // namespace pic
