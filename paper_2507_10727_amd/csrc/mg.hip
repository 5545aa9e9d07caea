// Geometric multigrid preconditioner and conjugate-gradient kernels of the
// FP32 inner solve (correction equation of the FP64 refinement).
//
// The operator is matrix-free: on a level with cell sizes dr, dz the
// couplings of the charge-form R-Z finite volumes, divided by 2 pi eps0, are
//   east  face (i+1/2, j): (i + 1/2) hz_j,  hz_j = dz (dz/2 on the z walls),
//   north face (i, j+1/2): g_i dr^2 / dz,   g_0 = 1/8, g_i = i, g_nr = nr/2 - 1/8,
// i.e. the face areas of the clipped control volumes over their spacings
// (Section 3's Gauss's law on the axis is the missing face at r = 0).
// Dirichlet nodes (anode row, outer column, cathode nodes of z = 0) carry a
// zero correction.
//
// One V-cycle is: per fine level a "down" kernel (MG_NU red-black
// Gauss-Seidel pairs from a zero guess, residual, full-weighting restriction
// of the residual, all in one LDS tile with a 1 + 2 MG_NU node halo), one
// single-workgroup "tail" kernel that runs every remaining coarse level in
// LDS and solves the coarsest with a dense inverse, and per fine level an
// "up" kernel (bilinear prolongation, MG_NU black-red pairs, 2 MG_NU node
// halo).  MG_NU = 1: with two pairs the CG iterations of a warm-started step
// drop from 6 to 5 but each V-cycle costs more, so it does not pay.  Pre-smoothing red-black and
// post-smoothing black-red with restriction = prolongation^T make the
// preconditioner symmetric, as conjugate gradients requires.
#include <cstring>

#include "common.h"

namespace pic {

namespace {

// bilinear prolongation of the coarse correction to fine node (i, j)
__device__ __forceinline__ float mg_prolong(const float *xc, int ldc, int i, int j)
{
    const int I = i >> 1, J = j >> 1;
    const float *c = xc + (int64_t)J * ldc + I;
    if (!(i & 1) && !(j & 1)) return c[0];
    if ((i & 1) && !(j & 1)) return 0.5f * (c[0] + c[1]);
    if (!(i & 1) && (j & 1)) return 0.5f * (c[0] + c[ldc]);
    return 0.25f * (c[0] + c[1] + c[ldc] + c[ldc + 1]);
}

// red-black Gauss-Seidel pairs before (red, black) and after (black, red)
// the coarse correction on every level; a half sweep is exact one node
// further inside the tile than the one before it, so the tiles carry halos
// of 1 + 2 MG_NU (down) and 2 MG_NU (up) fine nodes
constexpr int MG_NU = 1;
constexpr int DTX = 16, DTY = 8;                 // coarse nodes per down tile
constexpr int DH = 1 + 2 * MG_NU;
constexpr int DLW = 2 * DTX + 2 * DH - 1, DLH = 2 * DTY + 2 * DH - 1;
constexpr int UTX = 32, UTY = 16;                // fine nodes per up tile
constexpr int UH = 2 * MG_NU;
constexpr int ULW = UTX + 2 * UH, ULH = UTY + 2 * UH;

// Down: pre-smooth from zero, residual, restriction.  F.b is the fine
// right-hand side; writes the smoothed F.xd and the coarse C.b.
__device__ __forceinline__ void mg_down_body(const MGLevel &F, const MGLevel &C, int bx, int by)
{
    if (F.gate && *F.gate) return;
    __shared__ float sb[DLH][DLW];
    __shared__ float sx[DLH][DLW];
    const int I0 = bx * DTX, J0 = by * DTY;
    const int fi0 = 2 * I0 - DH, fj0 = 2 * J0 - DH;
    const int ld = F.nr + 1;
    for (int t = threadIdx.x; t < DLW * DLH; t += 256) {
        const int li = t % DLW, lj = t / DLW;
        const int i = fi0 + li, j = fj0 + lj;
        float bv = 0.0f, xv = 0.0f;
        if (mg_in(F, i, j) && mg_unknown(F, i, j)) {
            bv = F.b[(int64_t)j * ld + i];
            if (((i + j) & 1) == 0) {
                float w, e, s, n;
                mg_coup(F, i, j, w, e, s, n);
                xv = bv * __builtin_amdgcn_rcpf(w + e + s + n);
            }
        }
        sb[lj][li] = bv;
        sx[lj][li] = xv;
    }
    __syncthreads();
    // half sweeps k = 1 .. 2 MG_NU - 1 (black, red, ...) on the region k
    // nodes inside the tile
    for (int k = 1; k < 2 * MG_NU; ++k) {
        const int w_ = DLW - 2 * k, h_ = DLH - 2 * k, c = k & 1;
        for (int t = threadIdx.x; t < w_ * h_; t += 256) {
            const int li = k + t % w_, lj = k + t / w_;
            const int i = fi0 + li, j = fj0 + lj;
            if (((i + j) & 1) != c || !mg_in(F, i, j) || !mg_unknown(F, i, j)) continue;
            float w, e, s, n;
            mg_coup(F, i, j, w, e, s, n);
            const float off = w * sx[lj][li - 1] + e * sx[lj][li + 1] + s * sx[lj - 1][li] +
                              n * sx[lj + 1][li];
            sx[lj][li] = (sb[lj][li] + off) * __builtin_amdgcn_rcpf(w + e + s + n);
        }
        __syncthreads();
    }
    // residual on the region the restriction reads (written over b)
    for (int t = threadIdx.x; t < (DLW - 4 * MG_NU) * (DLH - 4 * MG_NU); t += 256) {
        const int li = 2 * MG_NU + t % (DLW - 4 * MG_NU), lj = 2 * MG_NU + t / (DLW - 4 * MG_NU);
        const int i = fi0 + li, j = fj0 + lj;
        float r = 0.0f;
        if (mg_in(F, i, j) && mg_unknown(F, i, j)) {
            float w, e, s, n;
            mg_coup(F, i, j, w, e, s, n);
            const float ax = (w + e + s + n) * sx[lj][li] -
                             (w * sx[lj][li - 1] + e * sx[lj][li + 1] + s * sx[lj - 1][li] +
                              n * sx[lj + 1][li]);
            r = sb[lj][li] - ax;
        }
        sb[lj][li] = r;
    }
    __syncthreads();
    const int ldc = C.nr + 1;
    for (int t = threadIdx.x; t < DTX * DTY; t += 256) {
        const int I = I0 + t % DTX, J = J0 + t / DTX;
        if (I > C.nr || J > C.nz) continue;
        float v = 0.0f;
        if (mg_unknown(C, I, J)) {
            const int ci = 2 * I - fi0, cj = 2 * J - fj0;
            v = sb[cj][ci] + 0.5f * (sb[cj][ci - 1] + sb[cj][ci + 1] + sb[cj - 1][ci] +
                                     sb[cj + 1][ci]) +
                0.25f * (sb[cj - 1][ci - 1] + sb[cj - 1][ci + 1] + sb[cj + 1][ci - 1] +
                         sb[cj + 1][ci + 1]);
        }
        C.b[(int64_t)J * ldc + I] = v;
    }
    // fine nodes owned by this tile: [2 I0, 2 I0 + 2 DTX) x [2 J0, 2 J0 + 2 DTY)
    for (int t = threadIdx.x; t < 4 * DTX * DTY; t += 256) {
        const int i = 2 * I0 + t % (2 * DTX), j = 2 * J0 + t / (2 * DTX);
        if (i > F.nr || j > F.nz) continue;
        F.xd[(int64_t)j * ld + i] = sx[j - fj0][i - fi0];
    }
}

// Up: x = xd + P xc, black then red Gauss-Seidel; writes F.xu on the owned
// tile and, if dot != null, accumulates sum(b * x) over it.
__device__ __forceinline__ void mg_up_body(const MGLevel &F, const MGLevel &C, double *dot, int bx,
                                           int by)
{
    if (F.gate && *F.gate) return;
    __shared__ float sb[ULH][ULW];
    __shared__ float sx[ULH][ULW];
    __shared__ double red[4];
    const int i0 = bx * UTX, j0 = by * UTY;
    const int fi0 = i0 - UH, fj0 = j0 - UH;
    const int ld = F.nr + 1, ldc = C.nr + 1;
    for (int t = threadIdx.x; t < ULW * ULH; t += 256) {
        const int li = t % ULW, lj = t / ULW;
        const int i = fi0 + li, j = fj0 + lj;
        float bv = 0.0f, xv = 0.0f;
        if (mg_in(F, i, j) && mg_unknown(F, i, j)) {
            const int64_t n = (int64_t)j * ld + i;
            bv = F.b[n];
            xv = F.xd[n] + mg_prolong(C.xu, ldc, i, j);
        }
        sb[lj][li] = bv;
        sx[lj][li] = xv;
    }
    __syncthreads();
    // half sweeps k = 0 .. 2 MG_NU - 1 (black, red, ...) on the region k + 1
    // nodes inside the tile
    for (int k = 0; k < 2 * MG_NU; ++k) {
        const int w_ = ULW - 2 * (k + 1), h_ = ULH - 2 * (k + 1), c = (k & 1) ? 0 : 1;
        for (int t = threadIdx.x; t < w_ * h_; t += 256) {
            const int li = k + 1 + t % w_, lj = k + 1 + t / w_;
            const int i = fi0 + li, j = fj0 + lj;
            if (((i + j) & 1) != c || !mg_in(F, i, j) || !mg_unknown(F, i, j)) continue;
            float w, e, s, n;
            mg_coup(F, i, j, w, e, s, n);
            const float off = w * sx[lj][li - 1] + e * sx[lj][li + 1] + s * sx[lj - 1][li] +
                              n * sx[lj + 1][li];
            sx[lj][li] = (sb[lj][li] + off) * __builtin_amdgcn_rcpf(w + e + s + n);
        }
        __syncthreads();
    }
    double acc = 0.0;
    for (int t = threadIdx.x; t < UTX * UTY; t += 256) {
        const int i = i0 + t % UTX, j = j0 + t / UTX;
        if (i > F.nr || j > F.nz) continue;
        const float v = sx[j - fj0][i - fi0];
        F.xu[(int64_t)j * ld + i] = v;
        acc += (double)v * (double)sb[j - fj0][i - fi0];
    }
    if (dot) {
        acc = wave_sum(acc);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
        __syncthreads();
        if (threadIdx.x == 0) {
            const double s = red[0] + red[1] + red[2] + red[3];
            if (s != 0.0) atomic_add_dev(dot, s);
        }
    }
}

// Tail: every level from `first` down to the coarsest in one workgroup
// (32 x 32 threads, thread (tx, ty) visits nodes i = tx + 32a, j = ty + 32b;
// a colour sweep visits only its own parity).  Reads L[first].b, writes
// L[first].xu (and sum(b * x) into dot if given).
constexpr int TT = 32;

__device__ __forceinline__ void tail_sweep(const MGLevel &L, float *x, const float *b, int c)
{
    const int ld = L.nr + 1;
    for (int j = threadIdx.y; j < L.nz; j += TT) {
        for (int i = 2 * threadIdx.x + ((j + c) & 1); i < L.nr; i += 2 * TT) {
            if (j == 0 && i < L.cath) continue;
            const int n = j * ld + i;
            float w, e, s, nn;
            mg_coup(L, i, j, w, e, s, nn);
            const float o = (i > 0 ? w * x[n - 1] : 0.0f) + e * x[n + 1] +
                            (j > 0 ? s * x[n - ld] : 0.0f) + nn * x[n + ld];
            x[n] = (b[n] + o) * __builtin_amdgcn_rcpf(w + e + s + nn);
        }
    }
}

__device__ __forceinline__ void mg_tail_body(const MGTail &T, double *dot, float *sm)
{
    if (T.L[T.first].gate && *T.L[T.first].gate) return;
    float *tmp = sm;
#define X(l) (sm + T.offx[(l)])
#define B(l) (sm + T.offb[(l)])
    const int tx = threadIdx.x, ty = threadIdx.y;
    {
        const MGLevel &L = T.L[T.first];
        const int ld = L.nr + 1;
        for (int j = ty; j <= L.nz; j += TT)
            for (int i = tx; i <= L.nr; i += TT) {
                const int n = j * ld + i;
                B(T.first)[n] = L.b[n];
                X(T.first)[n] = 0.0f;
            }
    }
    __syncthreads();
    // descend: x = 0, red-black sweep, residual, restriction
    for (int l = T.first; l < T.last; ++l) {
        const MGLevel &L = T.L[l];
        const int ld = L.nr + 1;
        float *x = X(l), *b = B(l);
        for (int k = 0; k < MG_NU; ++k) {
            tail_sweep(L, x, b, 0);
            __syncthreads();
            tail_sweep(L, x, b, 1);
            __syncthreads();
        }
        for (int j = ty; j <= L.nz; j += TT)
            for (int i = tx; i <= L.nr; i += TT) {
                const int n = j * ld + i;
                float r = 0.0f;
                if (mg_unknown(L, i, j)) {
                    float w, e, s, nn;
                    mg_coup(L, i, j, w, e, s, nn);
                    const float o = (i > 0 ? w * x[n - 1] : 0.0f) + e * x[n + 1] +
                                    (j > 0 ? s * x[n - ld] : 0.0f) + nn * x[n + ld];
                    r = b[n] - ((w + e + s + nn) * x[n] - o);
                }
                tmp[n] = r;
            }
        __syncthreads();
        const MGLevel &C = T.L[l + 1];
        const int ldc = C.nr + 1;
        for (int J = ty; J <= C.nz; J += TT)
            for (int I = tx; I <= C.nr; I += TT) {
                float v = 0.0f;
                if (mg_unknown(C, I, J)) {
                    const int c = 2 * J * ld + 2 * I;
                    const bool w = I > 0, s = J > 0;   // fine 2I-1 / 2J-1 exist
                    v = tmp[c] + 0.5f * ((w ? tmp[c - 1] : 0.0f) + tmp[c + 1] +
                                         (s ? tmp[c - ld] : 0.0f) + tmp[c + ld]) +
                        0.25f * ((w && s ? tmp[c - ld - 1] : 0.0f) + (s ? tmp[c - ld + 1] : 0.0f) +
                                 (w ? tmp[c + ld - 1] : 0.0f) + tmp[c + ld + 1]);
                }
                B(l + 1)[J * ldc + I] = v;
                X(l + 1)[J * ldc + I] = 0.0f;
            }
        __syncthreads();
    }
    // coarsest: dense inverse on the unknowns, x = A^-1 b; 32 lanes per row
    // (each a strided part of the row, summed with lane shuffles), so every
    // thread has only a few independent loads of the inverse in flight
    {
        const int tid = ty * TT + tx;
        const int g = tid >> 5, lane = tid & 31;
        const float *bc = B(T.last);
        for (int a0 = 0; a0 < T.ninv; a0 += (TT * TT) / 32) {
            const int a = a0 + g;
            float acc = 0.0f;
            if (a < T.ninv) {
                const float *row = T.inv + (int64_t)a * T.ninv;
                for (int c = lane; c < T.ninv; c += 32) acc += row[c] * bc[T.map[c]];
            }
            for (int o = 16; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 32);
            if (a < T.ninv && lane == 0) X(T.last)[T.map[a]] = acc;
        }
        __syncthreads();
    }
    // ascend: prolongation, black-red sweep
    for (int l = T.last - 1; l >= T.first; --l) {
        const MGLevel &L = T.L[l];
        const int ld = L.nr + 1, ldc = T.L[l + 1].nr + 1;
        float *x = X(l), *b = B(l);
        for (int j = ty; j <= L.nz; j += TT)
            for (int i = tx; i <= L.nr; i += TT)
                if (mg_unknown(L, i, j)) x[j * ld + i] += mg_prolong(X(l + 1), ldc, i, j);
        __syncthreads();
        for (int k = 0; k < MG_NU; ++k) {
            tail_sweep(L, x, b, 1);
            __syncthreads();
            tail_sweep(L, x, b, 0);
            __syncthreads();
        }
    }
    {
        const MGLevel &L = T.L[T.first];
        const int ld = L.nr + 1;
        double acc = 0.0;
        for (int j = ty; j <= L.nz; j += TT)
            for (int i = tx; i <= L.nr; i += TT) {
                const int n = j * ld + i;
                L.xu[n] = X(T.first)[n];
                acc += (double)X(T.first)[n] * (double)B(T.first)[n];
            }
        if (dot) {
            __shared__ double red[16];
            const int tid = ty * TT + tx;
            acc = wave_sum(acc);
            if ((tid & 63) == 0) red[tid >> 6] = acc;
            __syncthreads();
            if (tid == 0) {
                double s = 0.0;
                for (int w = 0; w < (TT * TT) / 64; ++w) s += red[w];
                if (s != 0.0) atomic_add_dev(dot, s);
            }
        }
    }
#undef X
#undef B
}

// ---- conjugate-gradient vector kernels on the finest level
constexpr int CB = 1024;   // CG vector kernels: few large blocks (one FP64 atomic each)

// p_k = z + beta p_{k-1} (beta = rz_k / rz_{k-1}, 0 for k = 0) into pc,
// q = A p_k, and p_k . q accumulated.
__device__ __forceinline__ void cg_matvec_body(const MGLevel &L, const float *z, const float *pp,
                                               float *pc, float *q, const double *rz, int k,
                                               double *pq, const double *zq, int blk, int nblk)
{
    if (L.gate && *L.gate) return;
    __shared__ double red[CB / 64];
    // Fletcher-Reeves beta for a fixed preconditioner; with zq (z_k.q_{k-1})
    // the Polak-Ribiere beta of flexible CG, z_k.(r_k - r_{k-1}) / z_{k-1}.r_{k-1}
    // = -z_k.q_{k-1} / p_{k-1}.q_{k-1}
    double bd = 0.0;
    if (zq) bd = (k > 0 && pq[-1] != 0.0) ? -zq[k] / pq[-1] : 0.0;
    else bd = (k > 0 && rz[k - 1] != 0.0) ? rz[k] / rz[k - 1] : 0.0;
    const float beta = (float)bd;
    const int ld = L.nr + 1;
    const int64_t nn = (int64_t)ld * (L.nz + 1);
    double acc = 0.0;
    for (int64_t n = (int64_t)blk * CB + threadIdx.x; n < nn; n += (int64_t)nblk * CB) {
        int i, j;
        node_ij(n, ld, i, j);
        float pv = 0.0f, qv = 0.0f;
        if (mg_unknown(L, i, j)) {
            float w, e, s, nb;
            mg_coup(L, i, j, w, e, s, nb);
            pv = z[n] + beta * pp[n];
            const float pe = z[n + 1] + beta * pp[n + 1];
            const float pnn = z[n + ld] + beta * pp[n + ld];
            const float pw = (i > 0) ? z[n - 1] + beta * pp[n - 1] : 0.0f;
            const float ps = (j > 0) ? z[n - ld] + beta * pp[n - ld] : 0.0f;
            qv = (w + e + s + nb) * pv - (w * pw + e * pe + s * ps + nb * pnn);
            acc += (double)pv * (double)qv;
        }
        pc[n] = pv;
        q[n] = qv;
    }
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < CB / 64; ++w) s += red[w];
        if (s != 0.0) atomic_add_dev(pq, s);
    }
}

// e += alpha p, r -= alpha q, ||r||^2 accumulated (alpha = rz_k / pq_k).
__device__ __forceinline__ void cg_update_body(int64_t nn, const float *p, const float *q, float *e,
                                               float *r, const double *rz, const double *pq,
                                               double *rr, const int32_t *gate, int blk, int nblk)
{
    if (gate && *gate) return;
    __shared__ double red[CB / 64];
    const float alpha = (*pq != 0.0) ? (float)(*rz / *pq) : 0.0f;
    double acc = 0.0;
    for (int64_t n = (int64_t)blk * CB + threadIdx.x; n < nn; n += (int64_t)nblk * CB) {
        e[n] += alpha * p[n];
        const float v = r[n] - alpha * q[n];
        r[n] = v;
        acc += (double)v * (double)v;
    }
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < CB / 64; ++w) s += red[w];
        if (s != 0.0) atomic_add_dev(rr, s);
    }
}

__global__ void __launch_bounds__(256) k_mg_down(MGLevel F, MGLevel C)
{
    mg_down_body(F, C, blockIdx.x, blockIdx.y);
}

__global__ void __launch_bounds__(256) k_mg_up(MGLevel F, MGLevel C, double *dot)
{
    mg_up_body(F, C, dot, blockIdx.x, blockIdx.y);
}

__global__ void __launch_bounds__(1024) k_mg_tail(MGTail T, double *dot)
{
    extern __shared__ float sm[];
    mg_tail_body(T, dot, sm);
}

__global__ void __launch_bounds__(CB) k_cg_matvec(MGLevel L, const float *z, const float *pp,
                                                  float *pc, float *q, const double *rz, int k,
                                                  double *pq, const double *zq)
{
    cg_matvec_body(L, z, pp, pc, q, rz, k, pq, zq, blockIdx.x, gridDim.x);
}

__global__ void __launch_bounds__(CB) k_cg_update(int64_t nn, const float *p, const float *q,
                                                  float *e, float *r, const double *rz,
                                                  const double *pq, double *rr,
                                                  const int32_t *gate)
{
    cg_update_body(nn, p, q, e, r, rz, pq, rr, gate, blockIdx.x, gridDim.x);
}

// ---- batched forms: one launch for the level (or vector) of every run of a
// batch; a block finds its run from the block offsets
__global__ void __launch_bounds__(256) k_mg_down_b(BatchArgs a)
{
    const int r = batch_run(a);
    const MGHier &H = a.run[r]->f.mg;
    const MGLevel &C = H.lv[a.level + 1];
    const int lb = blockIdx.x - a.off[r], tx = (C.nr + 1 + DTX - 1) / DTX;
    mg_down_body(H.lv[a.level], C, lb % tx, lb / tx);
}

__global__ void __launch_bounds__(256) k_mg_up_b(BatchArgs a)
{
    const int r = batch_run(a);
    const RunSolve &R = *a.run[r];
    const MGLevel &F = R.f.mg.lv[a.level];
    const int lb = blockIdx.x - a.off[r], tx = (F.nr + 1 + UTX - 1) / UTX;
    mg_up_body(F, R.f.mg.lv[a.level + 1], a.level == 0 ? &R.sc->pcg_rz[a.k] : nullptr, lb % tx,
               lb / tx);
}

__global__ void __launch_bounds__(1024) k_mg_tail_b(BatchArgs a)
{
    extern __shared__ float sm[];
    const RunSolve &R = *a.run[blockIdx.x];
    mg_tail_body(R.f.mg.tail, R.f.mg.tail.first == 0 ? &R.sc->pcg_rz[a.k] : nullptr, sm);
}

__global__ void __launch_bounds__(CB) k_cg_matvec_b(BatchArgs a)
{
    const int r = batch_run(a);
    const RunSolve &R = *a.run[r];
    const int k = a.k;
    cg_matvec_body(R.f.mg.lv[0], R.f.mg.lv[0].xu, R.f.p32[(k + 1) & 1], R.f.p32[k & 1], R.f.q32,
                   R.sc->pcg_rz, k, &R.sc->pcg_pq[k], nullptr, blockIdx.x - a.off[r],
                   a.off[r + 1] - a.off[r]);
}

__global__ void __launch_bounds__(CB) k_cg_update_b(BatchArgs a)
{
    const int r = batch_run(a);
    const RunSolve &R = *a.run[r];
    const int k = a.k;
    const MGLevel &L = R.f.mg.lv[0];
    cg_update_body((int64_t)(L.nr + 1) * (L.nz + 1), R.f.p32[k & 1], R.f.q32, R.f.e32, L.b,
                   &R.sc->pcg_rz[k], &R.sc->pcg_pq[k], &R.sc->pcg_rr[k], L.gate,
                   blockIdx.x - a.off[r], a.off[r + 1] - a.off[r]);
}

inline int cg_blocks(int64_t n)
{
    int64_t b = (n + CB - 1) / CB;
    // at most one block per CU: each ends in an FP64 atomic on one address,
    // and those are serialized
    return (int)std::max<int64_t>(1, std::min<int64_t>(b, 256));
}

}  // namespace

void launch_mg_vcycle(const MGHier &H, double *dot, hipStream_t s)
{
    // down the grid levels
    for (int l = 0; l < H.tail.first; ++l) {
        const MGLevel &F = H.lv[l], &C = H.lv[l + 1];
        dim3 g((C.nr + 1 + DTX - 1) / DTX, (C.nz + 1 + DTY - 1) / DTY);
        hipLaunchKernelGGL(k_mg_down, g, dim3(256), 0, s, F, C);
    }
    hipLaunchKernelGGL(k_mg_tail, dim3(1), dim3(TT, TT), H.tail_lds_bytes, s, H.tail,
                       H.tail.first == 0 ? dot : nullptr);
    for (int l = H.tail.first - 1; l >= 0; --l) {
        const MGLevel &F = H.lv[l], &C = H.lv[l + 1];
        dim3 g((F.nr + 1 + UTX - 1) / UTX, (F.nz + 1 + UTY - 1) / UTY);
        hipLaunchKernelGGL(k_mg_up, g, dim3(256), 0, s, F, C, l == 0 ? dot : nullptr);
    }
}

void launch_cg_matvec(const MGHier &H, const float *z, const float *pp, float *pc, float *q,
                      const double *rz, int k, double *pq, const double *zq, hipStream_t s)
{
    const MGLevel &L = H.lv[0];
    const int64_t nn = (int64_t)(L.nr + 1) * (L.nz + 1);
    hipLaunchKernelGGL(k_cg_matvec, dim3(cg_blocks(nn)), dim3(CB), 0, s, L, z, pp, pc, q, rz, k, pq,
                       zq);
}

void launch_cg_update(const MGHier &H, const float *p, const float *q, float *e, float *r,
                      const double *rz, const double *pq, double *rr, hipStream_t s)
{
    const MGLevel &L = H.lv[0];
    const int64_t nn = (int64_t)(L.nr + 1) * (L.nz + 1);
    hipLaunchKernelGGL(k_cg_update, dim3(cg_blocks(nn)), dim3(CB), 0, s, nn, p, q, e, r, rz, pq,
                       rr, L.gate);
}

// ---- batched launches over the runs of a plan
namespace {
BatchArgs batch_args(const BatchPlan &P)
{
    BatchArgs a;
    memset(&a, 0, sizeof(a));
    a.nruns = P.nruns;
    for (int r = 0; r < P.nruns; ++r) a.run[r] = P.dev[r];
    return a;
}
}  // namespace

void launch_mg_vcycle_b(const BatchPlan &P, int k, hipStream_t s)
{
    BatchArgs a = batch_args(P);
    a.k = k;
    int lmax = 0, tail_lds = 0;
    for (int r = 0; r < P.nruns; ++r) {
        lmax = std::max(lmax, (int)P.host[r].tail.first);
        tail_lds = std::max(tail_lds, (int)P.host[r].tail_lds_bytes);
    }
    for (int l = 0; l < lmax; ++l) {
        a.level = l;
        a.off[0] = 0;
        for (int r = 0; r < P.nruns; ++r) {
            const MGHier &H = P.host[r];
            int nb = 0;
            if (l < H.tail.first)
                nb = ((H.lv[l + 1].nr + 1 + DTX - 1) / DTX) * ((H.lv[l + 1].nz + 1 + DTY - 1) / DTY);
            a.off[r + 1] = a.off[r] + nb;
        }
        if (a.off[P.nruns] > 0)
            hipLaunchKernelGGL(k_mg_down_b, dim3(a.off[P.nruns]), dim3(256), 0, s, a);
    }
    for (int r = 0; r <= P.nruns; ++r) a.off[r] = r;
    hipLaunchKernelGGL(k_mg_tail_b, dim3(P.nruns), dim3(TT, TT), tail_lds, s, a);
    for (int l = lmax - 1; l >= 0; --l) {
        a.level = l;
        a.off[0] = 0;
        for (int r = 0; r < P.nruns; ++r) {
            const MGHier &H = P.host[r];
            int nb = 0;
            if (l < H.tail.first)
                nb = ((H.lv[l].nr + 1 + UTX - 1) / UTX) * ((H.lv[l].nz + 1 + UTY - 1) / UTY);
            a.off[r + 1] = a.off[r] + nb;
        }
        if (a.off[P.nruns] > 0)
            hipLaunchKernelGGL(k_mg_up_b, dim3(a.off[P.nruns]), dim3(256), 0, s, a);
    }
}

void launch_cg_matvec_b(const BatchPlan &P, int k, hipStream_t s)
{
    BatchArgs a = batch_args(P);
    a.k = k;
    for (int r = 0; r < P.nruns; ++r)
        a.off[r + 1] = a.off[r] + cg_blocks((int64_t)(P.host[r].lv[0].nr + 1) * (P.host[r].lv[0].nz + 1));
    hipLaunchKernelGGL(k_cg_matvec_b, dim3(a.off[P.nruns]), dim3(CB), 0, s, a);
}

void launch_cg_update_b(const BatchPlan &P, int k, hipStream_t s)
{
    BatchArgs a = batch_args(P);
    a.k = k;
    for (int r = 0; r < P.nruns; ++r)
        a.off[r + 1] = a.off[r] + cg_blocks((int64_t)(P.host[r].lv[0].nr + 1) * (P.host[r].lv[0].nz + 1));
    hipLaunchKernelGGL(k_cg_update_b, dim3(a.off[P.nruns]), dim3(CB), 0, s, a);
}

// The attribute is per kernel, not per hierarchy: both tail kernels get the
// largest tail any hierarchy may have, so runs of different sizes in one
// process never launch above the limit another run set.
int mg_tail_setup(MGHier &H)
{
    if (H.tail_lds_bytes > MG_TAIL_LDS_MAX) return 1;
    int e = (int)hipFuncSetAttribute((const void *)k_mg_tail,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, MG_TAIL_LDS_MAX);
    e |= (int)hipFuncSetAttribute((const void *)k_mg_tail_b,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, MG_TAIL_LDS_MAX);
    return e;
}

}  // namespace pic
