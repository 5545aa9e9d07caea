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

// The coarse levels are latency-bound (a few dozen blocks each), so every
// kernel here issues all global loads of a phase before it uses the first
// one, and reads its gate only after the loads are in flight: a loop that
// loads and stores one element at a time waits one memory latency per
// element.

// ---- LDS tiles of one level (W x H nodes from (fi0, fj0)), shared by the
// one- and two-level kernels; NT threads per block

// red initial value of pre-smoothing from zero: x = b / diag on red nodes
__device__ __forceinline__ float down_red(const MGLevel &F, int i, int j, float bv)
{
    if (((i + j) & 1) != 0) return 0.0f;
    float w, e, s, n;
    mg_coup(F, i, j, w, e, s, n);
    return bv * __builtin_amdgcn_rcpf(w + e + s + n);
}

// Pre-smoothing after the red initial values: half sweeps k = 1 .. 2 MG_NU - 1
// (black, red, ...) on the region k nodes inside the tile, then the residual
// on the region 2 MG_NU inside, written over sb.  Every step ends in a
// barrier.
template <int W, int H, int NT>
__device__ __forceinline__ void tile_down_smooth(const MGLevel &F, int fi0, int fj0, float (*sb)[W],
                                                 float (*sx)[W])
{
    for (int k = 1; k < 2 * MG_NU; ++k) {
        const int w_ = W - 2 * k, h_ = H - 2 * k, c = k & 1;
        for (int t = threadIdx.x; t < w_ * h_; t += NT) {
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
    constexpr int RW = W - 4 * MG_NU, RH = H - 4 * MG_NU;
    for (int t = threadIdx.x; t < RW * RH; t += NT) {
        const int li = 2 * MG_NU + t % RW, lj = 2 * MG_NU + t / RW;
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
}

// full weighting of the fine residual in sb around tile position (ci, cj)
template <int W>
__device__ __forceinline__ float tile_restrict(const float (*sb)[W], int ci, int cj)
{
    return sb[cj][ci] + 0.5f * (sb[cj][ci - 1] + sb[cj][ci + 1] + sb[cj - 1][ci] + sb[cj + 1][ci]) +
           0.25f * (sb[cj - 1][ci - 1] + sb[cj - 1][ci + 1] + sb[cj + 1][ci - 1] +
                    sb[cj + 1][ci + 1]);
}

// Post-smoothing after the prolonged correction is in sx: half sweeps
// k = 0 .. 2 MG_NU - 1 (black, red, ...) on the region k + 1 nodes inside the
// tile, each ending in a barrier.
template <int W, int H, int NT>
__device__ __forceinline__ void tile_up_smooth(const MGLevel &F, int fi0, int fj0, float (*sb)[W],
                                               float (*sx)[W])
{
    for (int k = 0; k < 2 * MG_NU; ++k) {
        const int w_ = W - 2 * (k + 1), h_ = H - 2 * (k + 1), c = (k & 1) ? 0 : 1;
        for (int t = threadIdx.x; t < w_ * h_; t += NT) {
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
}

// Loads of an up tile's unknown nodes: b, xd and the (up to four) coarse
// values of C.xu the bilinear prolongation reads: the east one only for odd
// i, the north one only for odd j (both exist there: a fine level has even nr
// and nz); the others, and the nodes that are not unknowns, load a node's own
// (or the first) value again.
template <int W, int H, int NT, int N>
__device__ __forceinline__ void up_loads(const MGLevel &F, const MGLevel &C, int fi0, int fj0,
                                         float *bl, float *xl, float *c0, float *c1, float *c2,
                                         float *c3)
{
    const int ld = F.nr + 1, ldc = C.nr + 1;
#pragma unroll
    for (int u = 0; u < N; ++u) {
        const int t = threadIdx.x + NT * u;
        const int i = fi0 + t % W, j = fj0 + t / W;
        const bool un = t < W * H && mg_in(F, i, j) && mg_unknown(F, i, j);
        const int64_t n = un ? (int64_t)j * ld + i : 0;
        const int64_t c = un ? (int64_t)(j >> 1) * ldc + (i >> 1) : 0;
        const int oi = un ? (i & 1) : 0, oj = un ? (j & 1) * ldc : 0;
        bl[u] = F.b[n];
        xl[u] = F.xd[n];
        c0[u] = C.xu[c];
        c1[u] = C.xu[c + oi];
        c2[u] = C.xu[c + oj];
        c3[u] = C.xu[c + oi + oj];
    }
}

// ---- one level per kernel

// Down: pre-smooth from zero, residual, restriction.  F.b is the fine
// right-hand side; writes the smoothed F.xd and the coarse C.b.
constexpr int DN = (DLW * DLH + 255) / 256;      // tile elements per thread (down)
constexpr int UN = (ULW * ULH + 255) / 256;      // (up)

__device__ __forceinline__ void mg_down_body(const MGLevel &F, const MGLevel &C, int bx, int by)
{
    const int32_t gated = gate_load(F.gate);
    __shared__ float sb[DLH][DLW];
    __shared__ float sx[DLH][DLW];
    const int I0 = bx * DTX, J0 = by * DTY;
    const int fi0 = 2 * I0 - DH, fj0 = 2 * J0 - DH;
    const int ld = F.nr + 1;
    float bl[DN];
#pragma unroll
    for (int u = 0; u < DN; ++u) {
        const int t = threadIdx.x + 256 * u;
        const int i = fi0 + t % DLW, j = fj0 + t / DLW;
        const bool un = t < DLW * DLH && mg_in(F, i, j) && mg_unknown(F, i, j);
        bl[u] = F.b[un ? (int64_t)j * ld + i : 0];
    }
#pragma unroll
    for (int u = 0; u < DN; ++u) {
        const int t = threadIdx.x + 256 * u;
        if (t >= DLW * DLH) continue;
        const int li = t % DLW, lj = t / DLW;
        const int i = fi0 + li, j = fj0 + lj;
        const bool un = mg_in(F, i, j) && mg_unknown(F, i, j);
        sb[lj][li] = un ? bl[u] : 0.0f;
        sx[lj][li] = un ? down_red(F, i, j, bl[u]) : 0.0f;
    }
    if (gated) return;   // uniform: the whole block leaves before its first barrier
    __syncthreads();
    tile_down_smooth<DLW, DLH, 256>(F, fi0, fj0, sb, sx);
    const int ldc = C.nr + 1;
    for (int t = threadIdx.x; t < DTX * DTY; t += 256) {
        const int I = I0 + t % DTX, J = J0 + t / DTX;
        if (I > C.nr || J > C.nz) continue;
        C.b[(int64_t)J * ldc + I] = mg_unknown(C, I, J) ? tile_restrict<DLW>(sb, 2 * I - fi0, 2 * J - fj0) : 0.0f;
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
    const int32_t gated = gate_load(F.gate);
    __shared__ float sb[ULH][ULW];
    __shared__ float sx[ULH][ULW];
    __shared__ double red[4];
    const int i0 = bx * UTX, j0 = by * UTY;
    const int fi0 = i0 - UH, fj0 = j0 - UH;
    const int ld = F.nr + 1;
    float bl[UN], xl[UN], c0[UN], c1[UN], c2[UN], c3[UN];
    up_loads<ULW, ULH, 256, UN>(F, C, fi0, fj0, bl, xl, c0, c1, c2, c3);
#pragma unroll
    for (int u = 0; u < UN; ++u) {
        const int t = threadIdx.x + 256 * u;
        if (t >= ULW * ULH) continue;
        const int li = t % ULW, lj = t / ULW;
        const int i = fi0 + li, j = fj0 + lj;
        const bool un = mg_in(F, i, j) && mg_unknown(F, i, j);
        sb[lj][li] = un ? bl[u] : 0.0f;
        sx[lj][li] = un ? xl[u] + mg_prolong_sel(i & 1, j & 1, c0[u], c1[u], c2[u], c3[u]) : 0.0f;
    }
    if (gated) return;
    __syncthreads();
    tile_up_smooth<ULW, ULH, 256>(F, fi0, fj0, sb, sx);
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

// ---- two levels per kernel (F -> M -> C down, C -> M -> F up), for the
// small grid levels just above the tail: one launch in place of two.  A tile
// carries the halos of both levels, and every node is computed with the
// operations of the one-level kernels (results agree to FP32 rounding: the
// compiler may contract multiply-adds differently in the two kernels).

// Down: tile of D2W x D2H coarse (C) nodes; the M region is what a one-level
// down tile of that size loads, the F region what the M region's b needs.
constexpr int D2W = 8, D2H = 4, D2T = 512;
constexpr int D2MW = 2 * D2W + 2 * DH - 1, D2MH = 2 * D2H + 2 * DH - 1;
constexpr int D2FW = 2 * D2MW + 2 * DH - 1, D2FH = 2 * D2MH + 2 * DH - 1;
constexpr int D2N = (D2FW * D2FH + D2T - 1) / D2T;

__device__ __forceinline__ void mg_down2_body(const MGLevel &F, const MGLevel &M, const MGLevel &C,
                                              int bx, int by)
{
    const int32_t gated = gate_load(F.gate);
    __shared__ float fb[D2FH][D2FW], fx[D2FH][D2FW];
    __shared__ float mb[D2MH][D2MW], mx[D2MH][D2MW];
    const int I0 = bx * D2W, J0 = by * D2H;
    const int mi0 = 2 * I0 - DH, mj0 = 2 * J0 - DH;
    const int fi0 = 2 * mi0 - DH, fj0 = 2 * mj0 - DH;
    const int ld = F.nr + 1, ldm = M.nr + 1, ldc = C.nr + 1;
    float bl[D2N];
#pragma unroll
    for (int u = 0; u < D2N; ++u) {
        const int t = threadIdx.x + D2T * u;
        const int i = fi0 + t % D2FW, j = fj0 + t / D2FW;
        const bool un = t < D2FW * D2FH && mg_in(F, i, j) && mg_unknown(F, i, j);
        bl[u] = F.b[un ? (int64_t)j * ld + i : 0];
    }
#pragma unroll
    for (int u = 0; u < D2N; ++u) {
        const int t = threadIdx.x + D2T * u;
        if (t >= D2FW * D2FH) continue;
        const int li = t % D2FW, lj = t / D2FW;
        const int i = fi0 + li, j = fj0 + lj;
        const bool un = mg_in(F, i, j) && mg_unknown(F, i, j);
        fb[lj][li] = un ? bl[u] : 0.0f;
        fx[lj][li] = un ? down_red(F, i, j, bl[u]) : 0.0f;
    }
    if (gated) return;
    __syncthreads();
    tile_down_smooth<D2FW, D2FH, D2T>(F, fi0, fj0, fb, fx);
    // M region: b restricted from F's residual, red initial x; the M nodes
    // this block owns ([2 I0, 2 I0 + 2 D2W) x [2 J0, 2 J0 + 2 D2H)) store b
    for (int t = threadIdx.x; t < D2MW * D2MH; t += D2T) {
        const int li = t % D2MW, lj = t / D2MW;
        const int I = mi0 + li, J = mj0 + lj;
        const bool un = mg_in(M, I, J) && mg_unknown(M, I, J);
        const float bv = un ? tile_restrict<D2FW>(fb, 2 * I - fi0, 2 * J - fj0) : 0.0f;
        mb[lj][li] = bv;
        mx[lj][li] = un ? down_red(M, I, J, bv) : 0.0f;
        if (I >= 2 * I0 && I < 2 * I0 + 2 * D2W && J >= 2 * J0 && J < 2 * J0 + 2 * D2H &&
            I <= M.nr && J <= M.nz)
            M.b[(int64_t)J * ldm + I] = bv;
    }
    // F nodes owned: [4 I0, 4 I0 + 4 D2W) x [4 J0, 4 J0 + 4 D2H)
    for (int t = threadIdx.x; t < 16 * D2W * D2H; t += D2T) {
        const int i = 4 * I0 + t % (4 * D2W), j = 4 * J0 + t / (4 * D2W);
        if (i > F.nr || j > F.nz) continue;
        F.xd[(int64_t)j * ld + i] = fx[j - fj0][i - fi0];
    }
    __syncthreads();
    tile_down_smooth<D2MW, D2MH, D2T>(M, mi0, mj0, mb, mx);
    for (int t = threadIdx.x; t < D2W * D2H; t += D2T) {
        const int I = I0 + t % D2W, J = J0 + t / D2W;
        if (I > C.nr || J > C.nz) continue;
        C.b[(int64_t)J * ldc + I] = mg_unknown(C, I, J) ? tile_restrict<D2MW>(mb, 2 * I - mi0, 2 * J - mj0) : 0.0f;
    }
    for (int t = threadIdx.x; t < 4 * D2W * D2H; t += D2T) {
        const int I = 2 * I0 + t % (2 * D2W), J = 2 * J0 + t / (2 * D2W);
        if (I > M.nr || J > M.nz) continue;
        M.xd[(int64_t)J * ldm + I] = mx[J - mj0][I - mi0];
    }
}

// Up: tile of UTX x UTY fine (F) nodes as in the one-level kernel; the M
// region covers the M nodes F's prolongation reads plus the M sweeps' halo.
constexpr int U2MW = UTX / 2 + 3 * UH + 1, U2MH = UTY / 2 + 3 * UH + 1;
constexpr int U2N = (U2MW * U2MH + 255) / 256;

__device__ __forceinline__ void mg_up2_body(const MGLevel &F, const MGLevel &M, const MGLevel &C,
                                            int bx, int by)
{
    const int32_t gated = gate_load(F.gate);
    __shared__ float fb[ULH][ULW], fx[ULH][ULW];
    __shared__ float mb[U2MH][U2MW], mx[U2MH][U2MW];
    const int i0 = bx * UTX, j0 = by * UTY;
    const int fi0 = i0 - UH, fj0 = j0 - UH;
    const int mi0 = (fi0 >> 1) - UH, mj0 = (fj0 >> 1) - UH;
    const int ld = F.nr + 1;
    float mbl[U2N], mxl[U2N], c0[U2N], c1[U2N], c2[U2N], c3[U2N];
    up_loads<U2MW, U2MH, 256, U2N>(M, C, mi0, mj0, mbl, mxl, c0, c1, c2, c3);
    float fbl[UN], fxl[UN];
#pragma unroll
    for (int u = 0; u < UN; ++u) {
        const int t = threadIdx.x + 256 * u;
        const int i = fi0 + t % ULW, j = fj0 + t / ULW;
        const bool un = t < ULW * ULH && mg_in(F, i, j) && mg_unknown(F, i, j);
        const int64_t n = un ? (int64_t)j * ld + i : 0;
        fbl[u] = F.b[n];
        fxl[u] = F.xd[n];
    }
#pragma unroll
    for (int u = 0; u < U2N; ++u) {
        const int t = threadIdx.x + 256 * u;
        if (t >= U2MW * U2MH) continue;
        const int li = t % U2MW, lj = t / U2MW;
        const int I = mi0 + li, J = mj0 + lj;
        const bool un = mg_in(M, I, J) && mg_unknown(M, I, J);
        mb[lj][li] = un ? mbl[u] : 0.0f;
        mx[lj][li] = un ? mxl[u] + mg_prolong_sel(I & 1, J & 1, c0[u], c1[u], c2[u], c3[u]) : 0.0f;
    }
    if (gated) return;
    __syncthreads();
    tile_up_smooth<U2MW, U2MH, 256>(M, mi0, mj0, mb, mx);
    // F: xd plus the prolongation of M's smoothed values (exact on the M
    // region UH nodes inside, which holds every M node read here)
#pragma unroll
    for (int u = 0; u < UN; ++u) {
        const int t = threadIdx.x + 256 * u;
        if (t >= ULW * ULH) continue;
        const int li = t % ULW, lj = t / ULW;
        const int i = fi0 + li, j = fj0 + lj;
        float bv = 0.0f, xv = 0.0f;
        if (mg_in(F, i, j) && mg_unknown(F, i, j)) {
            const int oi = i & 1, oj = j & 1;
            const int mi = (i >> 1) - mi0, mj = (j >> 1) - mj0;
            bv = fbl[u];
            xv = fxl[u] + mg_prolong_sel(oi, oj, mx[mj][mi], mx[mj][mi + oi], mx[mj + oj][mi],
                                         mx[mj + oj][mi + oi]);
        }
        fb[lj][li] = bv;
        fx[lj][li] = xv;
    }
    __syncthreads();
    tile_up_smooth<ULW, ULH, 256>(F, fi0, fj0, fb, fx);
    for (int t = threadIdx.x; t < UTX * UTY; t += 256) {
        const int i = i0 + t % UTX, j = j0 + t / UTX;
        if (i > F.nr || j > F.nz) continue;
        F.xu[(int64_t)j * ld + i] = fx[j - fj0][i - fi0];
    }
}

// ---- the finest level with the CG vector work fused in

__device__ __forceinline__ double ld_vec(const double *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// scalars of CG iteration j (uniform over the grid): beta_j, alpha_j and
// p_j.q_j from the dots of the V-cycle that produced z_j
struct CgScalars {
    float alpha, beta;
    double pq;
};
__device__ __forceinline__ CgScalars cg_scalars(const CgVecs &v, int j)
{
    // the slotted dots: lane l reads slot l mod CG_SLOTS of each (vector
    // loads, which queue with the kernel's other loads; scalar loads of
    // values the previous kernel wrote miss the scalar cache one after
    // another), summed over the slots by a butterfly that leaves the same
    // sums in every lane; index j - 1 is clamped and its terms selected away
    // for j = 0
    const int sl = threadIdx.x & (CG_SLOTS - 1);
    const int jm = j > 0 ? j - 1 : 0;
    double rz = ld_vec(&v.acc[cg_acc_at(j, 0, sl)]), rzm = ld_vec(&v.acc[cg_acc_at(jm, 0, sl)]);
    double zaz = ld_vec(&v.acc[cg_acc_at(j, 1, sl)]), zq = ld_vec(&v.acc[cg_acc_at(j, 2, sl)]);
    const double pqm = ld_vec(&v.pq[jm]);
#pragma unroll
    for (int o = CG_SLOTS / 2; o > 0; o >>= 1) {
        rz += __shfl_xor(rz, o, CG_SLOTS);
        rzm += __shfl_xor(rzm, o, CG_SLOTS);
        zaz += __shfl_xor(zaz, o, CG_SLOTS);
        zq += __shfl_xor(zq, o, CG_SLOTS);
    }
    CgScalars c;
    const double bd = (j > 0 && rzm != 0.0) ? rz / rzm : 0.0;
    c.pq = zaz + (j > 0 ? 2.0 * bd * zq + bd * bd * pqm : 0.0);
    c.beta = (float)bd;
    c.alpha = (c.pq > 0.0) ? (float)(rz / c.pq) : 0.0f;
    return c;
}

// Down on the finest level with the update of CG iteration j applied first:
// the tile (halo included) forms q_j = w_j + beta q_{j-1} and r_{j+1} =
// r_j - alpha q_j from r[j & 1], w, q[(j - 1) & 1]; owned nodes store
// r[(j + 1) & 1], q[j & 1], p_j = z_j + beta p_{j-1} (in place), e += alpha
// p_j and add r_{j+1}^2 to their slot of ||r_{j+1}||^2; then pre-smoothing
// of r_{j+1} as in the plain down kernel.  Block (0, 0) records p_j.q_j in
// pq[j].
static_assert(MG_NU >= 1, "the owned-node pass reads sb before the smoothing's first barrier");
__device__ __forceinline__ void mg_down_cg_body(const MGLevel &F, const MGLevel &C,
                                                const CgVecs &v, int j, int bx, int by)
{
    __shared__ float sb[DLH][DLW], sx[DLH][DLW], sq[DLH][DLW];
    __shared__ double red[4];
    const int I0 = bx * DTX, J0 = by * DTY;
    const int fi0 = 2 * I0 - DH, fj0 = 2 * J0 - DH;
    const int ld = F.nr + 1;
    const float *rold = v.r[j & 1], *qold = v.q[(j + 1) & 1];   // q_{j-1} (unused for j = 0)
    float rl[DN], wl[DN], ql[DN];
#pragma unroll
    for (int u = 0; u < DN; ++u) {
        const int t = threadIdx.x + 256 * u;
        const int i = fi0 + t % DLW, jj = fj0 + t / DLW;
        const bool un = t < DLW * DLH && mg_in(F, i, jj) && mg_unknown(F, i, jj);
        const int64_t n = un ? (int64_t)jj * ld + i : 0;
        rl[u] = rold[n];
        wl[u] = v.w[n];
        ql[u] = qold[n];
    }
    // owned nodes [2 I0, 2 I0 + 2 DTX) x [2 J0, 2 J0 + 2 DTY): z, p_{j-1}, e
    constexpr int ON = (4 * DTX * DTY + 255) / 256;
    float zl[ON], pl[ON], el[ON];
#pragma unroll
    for (int o = 0; o < ON; ++o) {
        const int t = threadIdx.x + 256 * o;
        const int i = 2 * I0 + t % (2 * DTX), jj = 2 * J0 + t / (2 * DTX);
        const int64_t n = (i <= F.nr && jj <= F.nz) ? (int64_t)jj * ld + i : 0;
        zl[o] = F.xu[n];
        pl[o] = v.p[n];
        el[o] = v.e[n];
    }
    // issued after the tile's loads: they complete in order, so the scalars'
    // wait is the tile's
    const int32_t gated = gate_load(F.gate);
    const CgScalars cs = cg_scalars(v, j);
    if (gated) return;   // uniform: the whole block leaves before its first barrier
#pragma unroll
    for (int u = 0; u < DN; ++u) {
        const int t = threadIdx.x + 256 * u;
        if (t >= DLW * DLH) continue;
        const int li = t % DLW, lj = t / DLW;
        const int i = fi0 + li, jj = fj0 + lj;
        const bool un = mg_in(F, i, jj) && mg_unknown(F, i, jj);
        const float qv = j > 0 ? wl[u] + cs.beta * ql[u] : wl[u];
        const float rn = rl[u] - cs.alpha * qv;
        sb[lj][li] = un ? rn : 0.0f;
        sx[lj][li] = un ? down_red(F, i, jj, rn) : 0.0f;
        sq[lj][li] = un ? qv : 0.0f;
    }
    __syncthreads();
    double acc = 0.0;
#pragma unroll
    for (int o = 0; o < ON; ++o) {
        const int t = threadIdx.x + 256 * o;
        const int i = 2 * I0 + t % (2 * DTX), jj = 2 * J0 + t / (2 * DTX);
        if (t >= 4 * DTX * DTY || i > F.nr || jj > F.nz) continue;
        const int64_t n = (int64_t)jj * ld + i;
        const float rn = sb[jj - fj0][i - fi0];
        const float pv = j > 0 ? zl[o] + cs.beta * pl[o] : zl[o];
        v.p[n] = pv;
        v.e[n] = el[o] + cs.alpha * pv;
        v.q[j & 1][n] = sq[jj - fj0][i - fi0];
        v.r[(j + 1) & 1][n] = rn;
        acc += (double)rn * (double)rn;
    }
    if (bx == 0 && by == 0 && threadIdx.x == 0) v.pq[j] = cs.pq;
    tile_down_smooth<DLW, DLH, 256>(F, fi0, fj0, sb, sx);
    const int ldc = C.nr + 1;
    for (int t = threadIdx.x; t < DTX * DTY; t += 256) {
        const int I = I0 + t % DTX, J = J0 + t / DTX;
        if (I > C.nr || J > C.nz) continue;
        C.b[(int64_t)J * ldc + I] = mg_unknown(C, I, J) ? tile_restrict<DLW>(sb, 2 * I - fi0, 2 * J - fj0) : 0.0f;
    }
    for (int t = threadIdx.x; t < 4 * DTX * DTY; t += 256) {
        const int i = 2 * I0 + t % (2 * DTX), jj = 2 * J0 + t / (2 * DTX);
        if (i > F.nr || jj > F.nz) continue;
        F.xd[(int64_t)jj * ld + i] = sx[jj - fj0][i - fi0];
    }
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        const double s = red[0] + red[1] + red[2] + red[3];
        const int sl = (by * (int)gridDim.x + bx) & (CG_SLOTS - 1);
        if (s != 0.0) atomic_add_dev(&v.acc[cg_acc_at(j, 3, sl)], s);
    }
}

// Up on the finest level of CG iteration k (F.b = r_k): a tile with one more
// halo node, so that after the sweeps z is exact on the owned nodes and their
// neighbours; owned nodes store z (F.xu) and w = A z, and the block adds
// r.z, z.w and z.q_{k-1} (k > 0) to its slot of iteration k's dots.
constexpr int UH3 = UH + 1;
constexpr int UCW = UTX + 2 * UH3, UCH = UTY + 2 * UH3;
constexpr int UCN = (UCW * UCH + 255) / 256;

__device__ __forceinline__ void mg_up_cg_body(const MGLevel &F, const MGLevel &C, const CgVecs &v,
                                              int k, int bx, int by)
{
    __shared__ float sb[UCH][UCW], sx[UCH][UCW];
    __shared__ double red[3][4];
    const int i0 = bx * UTX, j0 = by * UTY;
    const int fi0 = i0 - UH3, fj0 = j0 - UH3;
    const int ld = F.nr + 1;
    float bl[UCN], xl[UCN], c0[UCN], c1[UCN], c2[UCN], c3[UCN];
    up_loads<UCW, UCH, 256, UCN>(F, C, fi0, fj0, bl, xl, c0, c1, c2, c3);
    constexpr int ON = (UTX * UTY + 255) / 256;
    const float *qold = v.q[(k + 1) & 1];   // q_{k-1} (unused for k = 0)
    float ql[ON];
#pragma unroll
    for (int o = 0; o < ON; ++o) {
        const int t = threadIdx.x + 256 * o;
        const int i = i0 + t % UTX, jj = j0 + t / UTX;
        ql[o] = qold[(i <= F.nr && jj <= F.nz) ? (int64_t)jj * ld + i : 0];
    }
    const int32_t gated = gate_load(F.gate);
    if (gated) return;   // uniform: the whole block leaves before its first barrier
#pragma unroll
    for (int u = 0; u < UCN; ++u) {
        const int t = threadIdx.x + 256 * u;
        if (t >= UCW * UCH) continue;
        const int li = t % UCW, lj = t / UCW;
        const int i = fi0 + li, jj = fj0 + lj;
        const bool un = mg_in(F, i, jj) && mg_unknown(F, i, jj);
        sb[lj][li] = un ? bl[u] : 0.0f;
        sx[lj][li] = un ? xl[u] + mg_prolong_sel(i & 1, jj & 1, c0[u], c1[u], c2[u], c3[u]) : 0.0f;
    }
    __syncthreads();
    tile_up_smooth<UCW, UCH, 256>(F, fi0, fj0, sb, sx);
    double a_rz = 0.0, a_zaz = 0.0, a_zq = 0.0;
#pragma unroll
    for (int o = 0; o < ON; ++o) {
        const int t = threadIdx.x + 256 * o;
        const int i = i0 + t % UTX, jj = j0 + t / UTX;
        if (i > F.nr || jj > F.nz) continue;
        const int li = i - fi0, lj = jj - fj0;
        const float z = sx[lj][li];
        float w = 0.0f;
        if (mg_unknown(F, i, jj)) {
            float cw, ce, cs, cn;
            mg_coup(F, i, jj, cw, ce, cs, cn);
            w = (cw + ce + cs + cn) * z - (cw * sx[lj][li - 1] + ce * sx[lj][li + 1] +
                                            cs * sx[lj - 1][li] + cn * sx[lj + 1][li]);
        }
        const int64_t n = (int64_t)jj * ld + i;
        F.xu[n] = z;
        v.w[n] = w;
        a_rz += (double)z * (double)sb[lj][li];
        a_zaz += (double)z * (double)w;
        if (k > 0) a_zq += (double)z * (double)ql[o];
    }
    a_rz = wave_sum(a_rz);
    a_zaz = wave_sum(a_zaz);
    a_zq = wave_sum(a_zq);
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = a_rz;
        red[1][threadIdx.x >> 6] = a_zaz;
        red[2][threadIdx.x >> 6] = a_zq;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        const double s = red[threadIdx.x][0] + red[threadIdx.x][1] + red[threadIdx.x][2] +
                         red[threadIdx.x][3];
        const int sl = (by * (int)gridDim.x + bx) & (CG_SLOTS - 1);
        if (s != 0.0) atomic_add_dev(&v.acc[cg_acc_at(k, threadIdx.x, sl)], s);
    }
}

// Tail: every level from `first` down to the coarsest in one workgroup of
// TT x TT threads, all in LDS.  Reads L[first].b, writes L[first].xu (and
// sum(b * x) into dot if given).  Loops run flat over a level's nodes (or
// over one colour's nodes in a sweep); each pass of a thread issues all of
// its LDS reads before it uses them, and the couplings and the absent
// neighbours of boundary nodes are selected, not branched around, so a pass
// waits for LDS once.
constexpr int TT = 32;
constexpr int TN = TT * TT;

// Per-level constants, read from the kernel argument once per level and held
// in scalar registers (the compiler would otherwise re-read the invariant
// argument inside every loop and wait for each read).
struct TailLevel {
    int nr, nz, cath, ld;
    float dz, dr2dz;
    float rld, rhalf;           // 1 / ld and 1 / (nr / 2), for the node index split
    float *x, *b;
};

// q = n / d for the small counts of a tail level (0 <= n < 2^22, 0 < d), from
// the float reciprocal rd ~ 1 / d: the estimate is off by at most one, fixed
// with full-rate 24-bit multiplies (a 32-bit division costs quarter-rate
// multiplies, and the tail is instruction-bound on its one CU)
__device__ __forceinline__ int tail_div(int n, int d, float rd)
{
    int q = (int)((float)n * rd);
    const int r = n - __mul24(q, d);
    q += (r >= d) ? 1 : 0;
    q -= (r < 0) ? 1 : 0;
    return q;
}
__device__ __forceinline__ void tail_ij(int n, const TailLevel &L, int &i, int &j)
{
    j = tail_div(n, L.ld, L.rld);
    i = n - __mul24(j, L.ld);
}

// (the batched kernel reads the same fields from device memory into vector
// registers: readfirstlane moves the uniform value to a scalar register)
__device__ __forceinline__ int in_sreg(int v)
{
    int r = __builtin_amdgcn_readfirstlane(v);
    asm volatile("" : "+s"(r));
    return r;
}
__device__ __forceinline__ float in_sreg(float v)
{
    return __builtin_bit_cast(float, in_sreg(__builtin_bit_cast(int, v)));
}

__device__ __forceinline__ TailLevel tail_level(const MGTail &T, float *sm, int l)
{
    TailLevel v;
    v.nr = in_sreg(T.L[l].nr);
    v.nz = in_sreg(T.L[l].nz);
    v.cath = in_sreg(T.L[l].cath);
    v.ld = v.nr + 1;
    v.dz = in_sreg(T.L[l].dz);
    v.dr2dz = in_sreg(T.L[l].dr2dz);
    v.rld = __builtin_amdgcn_rcpf((float)v.ld);
    v.rhalf = __builtin_amdgcn_rcpf((float)(v.nr > 1 ? v.nr >> 1 : 1));
    v.x = sm + in_sreg(T.offx[l]);
    v.b = sm + in_sreg(T.offb[l]);
    return v;
}

__device__ __forceinline__ bool tail_unknown(const TailLevel &L, int i, int j)
{
    return i < L.nr && j < L.nz && !(j == 0 && i < L.cath);
}

// A x - b's negative at unknown node (i, j) = m: b - (diag x - sum c x_nb);
// the west / south neighbours of the first column / row read the node
// itself, with a zero coupling
__device__ __forceinline__ float tail_res(const TailLevel &L, int i, int j, int m)
{
    float w, e, s, n;
    mg_coup_v(L.nr, L.nz, L.dz, L.dr2dz, i, j, w, e, s, n);
    const float o = w * L.x[m - (i > 0 ? 1 : 0)] + e * L.x[m + 1] +
                    s * L.x[m - (j > 0 ? L.ld : 0)] + n * L.x[m + L.ld];
    return L.b[m] - ((w + e + s + n) * L.x[m] - o);
}

// One colour c of a red-black sweep: nodes with (i + j + c) even.  A swept
// level has even nr (it has a coarser level), so each row holds nr / 2 nodes
// of a colour.  One node per pass: the workgroup's 16 waves hide the LDS
// latency, and a second node per pass would only add instructions.
__device__ __forceinline__ void tail_sweep(const TailLevel &L, int c, int tid)
{
    const int half = L.nr >> 1, cnt = __mul24(half, L.nz);
    for (int h = tid; h < cnt; h += TN) {
        const int j = tail_div(h, half, L.rhalf);
        const int i = 2 * (h - __mul24(j, half)) + ((j + c) & 1);
        if (j == 0 && i < L.cath) continue;
        float w, e, s, n;
        mg_coup_v(L.nr, L.nz, L.dz, L.dr2dz, i, j, w, e, s, n);
        const int m = __mul24(j, L.ld) + i;
        const float o = w * L.x[m - (i > 0 ? 1 : 0)] + e * L.x[m + 1] +
                        s * L.x[m - (j > 0 ? L.ld : 0)] + n * L.x[m + L.ld];
        L.x[m] = (L.b[m] + o) * __builtin_amdgcn_rcpf(w + e + s + n);
    }
}

// Right-hand-side values per thread loaded up front, and the share of the
// dense inverse held in registers (rows g + 32 r, columns lane + 32 m of a
// 32-lane group g): inverses of up to 32 TDR unknowns are prefetched,
// larger ones read when needed.
constexpr int TBN = MG_TAIL_NODES_MAX / TN;
constexpr int TDR = 7;
static_assert(TBN * TN == MG_TAIL_NODES_MAX, "tail rows per thread");

__device__ __forceinline__ void mg_tail_body(const MGTail &T, double *dot, float *sm)
{
    const int32_t gated = gate_load(T.L[T.first].gate);
    float *tmp = sm;
    const int tid = threadIdx.y * TT + threadIdx.x;
    const int g = tid >> 5, lane = tid & 31;
    const bool dense_regs = T.ninv > 0 && T.ninv <= 32 * TDR;
    float bl[TBN], inv[TDR][TDR];
    int32_t col[TDR];
#pragma unroll
    for (int u = 0; u < TBN; ++u) {
        const int n = tid + TN * u;
        bl[u] = T.L[T.first].b[n < T.tmp_size ? n : 0];
    }
    {
        const TailLevel L = tail_level(T, sm, T.first);
#pragma unroll
        for (int u = 0; u < TBN; ++u) {
            const int n = tid + TN * u;
            if (n < T.tmp_size) {
                L.b[n] = bl[u];
                L.x[n] = 0.0f;
            }
        }
    }
    if (gated) return;   // uniform: the whole block leaves before its first barrier
    __syncthreads();
    // the inverse's share, issued once every wave has its right-hand side
    // (loads queue in order: ahead of them they would delay the first
    // phase), arrives while the levels above the coarsest are smoothed;
    // only the nb x nb blocks of 32 rows / columns the inverse has
    const int nb = dense_regs ? (T.ninv + 31) >> 5 : 0;
#pragma unroll
    for (int m = 0; m < TDR; ++m) {
        if (m >= nb) break;
        const int c = lane + 32 * m;
        col[m] = T.map[c < T.ninv ? c : 0];
#pragma unroll
        for (int r = 0; r < TDR; ++r) {
            if (r >= nb) break;
            const int a = g + 32 * r;
            inv[r][m] = T.inv[(c < T.ninv && a < T.ninv) ? (int64_t)a * T.ninv + c : 0];
        }
    }
    // descend: x = 0, red-black sweep, residual, restriction
    for (int l = T.first; l < T.last; ++l) {
        const TailLevel L = tail_level(T, sm, l);
        for (int k = 0; k < MG_NU; ++k) {
            tail_sweep(L, 0, tid);
            __syncthreads();
            tail_sweep(L, 1, tid);
            __syncthreads();
        }
        const int nn = L.ld * (L.nz + 1);
        for (int n = tid; n < nn; n += TN) {
            int i, j;
            tail_ij(n, L, i, j);
            tmp[n] = tail_unknown(L, i, j) ? tail_res(L, i, j, n) : 0.0f;
        }
        __syncthreads();
        const TailLevel C = tail_level(T, sm, l + 1);
        const int nc = C.ld * (C.nz + 1);
        for (int n = tid; n < nc; n += TN) {
            int I, J;
            tail_ij(n, C, I, J);
            float v = 0.0f;
            if (tail_unknown(C, I, J)) {
                // full weighting of the fine residual; fine nodes 2I-1 / 2J-1
                // are absent on the first coarse column / row
                const int c = 2 * J * L.ld + 2 * I;
                const bool w = I > 0, s = J > 0;
                const int dw = w ? 1 : 0, ds = s ? L.ld : 0;
                const float tw = tmp[c - dw], ts = tmp[c - ds], tsw = tmp[c - ds - dw];
                const float tse = tmp[c - ds + 1], tnw = tmp[c + L.ld - dw];
                v = tmp[c] + 0.5f * ((w ? tw : 0.0f) + tmp[c + 1] + (s ? ts : 0.0f) + tmp[c + L.ld]) +
                    0.25f * ((w && s ? tsw : 0.0f) + (s ? tse : 0.0f) + (w ? tnw : 0.0f) +
                             tmp[c + L.ld + 1]);
            }
            C.b[n] = v;
            C.x[n] = 0.0f;
        }
        __syncthreads();
    }
    // coarsest: dense inverse on the unknowns, x = A^-1 b; 32 lanes per row
    // (each a strided part of the row, summed with lane shuffles)
    {
        const TailLevel C = tail_level(T, sm, T.last);
        if (dense_regs) {
            float bq[TDR], acc[TDR];
#pragma unroll
            for (int m = 0; m < TDR; ++m) {
                if (m >= nb) break;
                bq[m] = C.b[col[m]];
            }
#pragma unroll
            for (int r = 0; r < TDR; ++r) {
                if (r >= nb) break;
                acc[r] = 0.0f;
#pragma unroll
                for (int m = 0; m < TDR; ++m) {
                    if (m >= nb) break;
                    if (lane + 32 * m < T.ninv) acc[r] += inv[r][m] * bq[m];
                }
            }
            // the rows' shuffle steps interleaved: one LDS wait per step
#pragma unroll
            for (int o = 16; o > 0; o >>= 1)
#pragma unroll
                for (int r = 0; r < TDR; ++r) {
                    if (r >= nb) break;
                    acc[r] += __shfl_xor(acc[r], o, 32);
                }
            // every lane holds the sums; lane g holds map[g + 32 r] = map[a]
#pragma unroll
            for (int r = 0; r < TDR; ++r) {
                if (r >= nb) break;
                if (g + 32 * r < T.ninv && lane == g) C.x[col[r]] = acc[r];
            }
        } else {
            for (int a0 = 0; a0 < T.ninv; a0 += TN / 32) {
                const int a = a0 + g;
                float acc = 0.0f;
                if (a < T.ninv) {
                    const float *row = T.inv + (int64_t)a * T.ninv;
                    for (int c = lane; c < T.ninv; c += 32) acc += row[c] * C.b[T.map[c]];
                }
                for (int o = 16; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 32);
                if (a < T.ninv && lane == 0) C.x[T.map[a]] = acc;
            }
        }
        __syncthreads();
    }
    // ascend: prolongation, black-red sweep
    for (int l = T.last - 1; l >= T.first; --l) {
        const TailLevel L = tail_level(T, sm, l);
        const TailLevel C = tail_level(T, sm, l + 1);
        const int nn = L.ld * (L.nz + 1);
        for (int n = tid; n < nn; n += TN) {
            int i, j;
            tail_ij(n, L, i, j);
            if (tail_unknown(L, i, j)) {
                // unknown fine nodes have i < nr, j < nz: the east / north
                // coarse values exist where odd i / j reads them
                const int oi = i & 1, oj = (j & 1) ? C.ld : 0;
                const float *c = C.x + (j >> 1) * C.ld + (i >> 1);
                L.x[n] += mg_prolong_sel(oi, oj, c[0], c[oi], c[oj], c[oi + oj]);
            }
        }
        __syncthreads();
        for (int k = 0; k < MG_NU; ++k) {
            tail_sweep(L, 1, tid);
            __syncthreads();
            tail_sweep(L, 0, tid);
            __syncthreads();
        }
    }
    {
        const TailLevel L = tail_level(T, sm, T.first);
        float *xu = T.L[T.first].xu;
        double acc = 0.0;
        for (int n = tid; n < T.tmp_size; n += TN) {
            const float v = L.x[n];
            xu[n] = v;
            acc += (double)v * (double)L.b[n];
        }
        if (dot) {
            __shared__ double red[TN / 64];
            acc = wave_sum(acc);
            if ((tid & 63) == 0) red[tid >> 6] = acc;
            __syncthreads();
            if (tid == 0) {
                double s = 0.0;
                for (int w = 0; w < TN / 64; ++w) s += red[w];
                if (s != 0.0) atomic_add_dev(dot, s);
            }
        }
    }
}

// ---- conjugate-gradient vector kernels on the finest level
constexpr int CB = 1024;   // CG vector kernels: few large blocks (one FP64 atomic each)

// p_k = z + beta p_{k-1} (beta = rz_k / rz_{k-1}, 0 for k = 0) into pc,
// q = A p_k, and p_k . q accumulated.
__device__ __forceinline__ void cg_matvec_body(const MGLevel &L, const float *z, const float *pp,
                                               float *pc, float *q, const double *rz, int k,
                                               double *pq, const double *zq, int blk, int nblk)
{
    const int32_t gated = gate_load(L.gate);   // tested after the loads are issued
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
        if (gated) return;
        pc[n] = pv;
        q[n] = qv;
    }
    if (gated) return;
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
    const int32_t gated = gate_load(gate);   // tested after the loads are issued
    __shared__ double red[CB / 64];
    const float alpha = (*pq != 0.0) ? (float)(*rz / *pq) : 0.0f;
    double acc = 0.0;
    for (int64_t n = (int64_t)blk * CB + threadIdx.x; n < nn; n += (int64_t)nblk * CB) {
        const float en = e[n] + alpha * p[n];
        const float v = r[n] - alpha * q[n];
        if (gated) return;
        e[n] = en;
        r[n] = v;
        acc += (double)v * (double)v;
    }
    if (gated) return;
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < CB / 64; ++w) s += red[w];
        if (s != 0.0) atomic_add_dev(rr, s);
    }
}

// The update of the last CG iteration j of a pass (no V-cycle follows):
// p_j, q_j, e += alpha p_j and ||r_{j+1}||^2 over all nodes.
__device__ __forceinline__ void cg_update_last_body(const MGLevel &L, const CgVecs &v, int j,
                                                    int blk, int nblk)
{
    __shared__ double red[CB / 64];
    const int32_t gated = gate_load(L.gate);
    const CgScalars cs = cg_scalars(v, j);
    if (gated) return;   // uniform: the whole block leaves before its first barrier
    const float *rold = v.r[j & 1], *qold = v.q[(j + 1) & 1];
    const int64_t nn = (int64_t)(L.nr + 1) * (L.nz + 1);
    double acc = 0.0;
    for (int64_t n = (int64_t)blk * CB + threadIdx.x; n < nn; n += (int64_t)nblk * CB) {
        const float w = v.w[n], z = L.xu[n], qo = qold[n], po = v.p[n], en = v.e[n], ro = rold[n];
        const float qv = j > 0 ? w + cs.beta * qo : w;
        const float pv = j > 0 ? z + cs.beta * po : z;
        v.e[n] = en + cs.alpha * pv;
        const float rn = ro - cs.alpha * qv;
        acc += (double)rn * (double)rn;
    }
    if (blk == 0 && threadIdx.x == 0) v.pq[j] = cs.pq;
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < CB / 64; ++w) s += red[w];
        if (s != 0.0) atomic_add_dev(&v.acc[cg_acc_at(j, 3, blk & (CG_SLOTS - 1))], s);
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

__global__ void __launch_bounds__(D2T) k_mg_down2(MGLevel F, MGLevel M, MGLevel C)
{
    mg_down2_body(F, M, C, blockIdx.x, blockIdx.y);
}

__global__ void __launch_bounds__(256) k_mg_up2(MGLevel F, MGLevel M, MGLevel C)
{
    mg_up2_body(F, M, C, blockIdx.x, blockIdx.y);
}

__global__ void __launch_bounds__(256) k_mg_down_cg(MGLevel F, MGLevel C, CgVecs v, int j)
{
    mg_down_cg_body(F, C, v, j, blockIdx.x, blockIdx.y);
}

__global__ void __launch_bounds__(256) k_mg_up_cg(MGLevel F, MGLevel C, CgVecs v, int k)
{
    mg_up_cg_body(F, C, v, k, blockIdx.x, blockIdx.y);
}

__global__ void __launch_bounds__(CB) k_cg_update_last(MGLevel L, CgVecs v, int j)
{
    cg_update_last_body(L, v, j, blockIdx.x, gridDim.x);
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

// fused forms: F.b of the finest level is r[k & 1] of the run's CG vectors
// (r[0] is the level's own b, so iteration 0 goes down with k_mg_down_b)
__global__ void __launch_bounds__(256) k_mg_down_cg_b(BatchArgs a)
{
    const int r = batch_run(a);
    const RunSolve &R = *a.run[r];
    MGLevel F = R.f.mg.lv[0];
    F.b = R.cg.r[a.k & 1];
    const MGLevel &C = R.f.mg.lv[1];
    const int lb = blockIdx.x - a.off[r], tx = (C.nr + 1 + DTX - 1) / DTX;
    mg_down_cg_body(F, C, R.cg, a.k - 1, lb % tx, lb / tx);
}

__global__ void __launch_bounds__(256) k_mg_up_cg_b(BatchArgs a)
{
    const int r = batch_run(a);
    const RunSolve &R = *a.run[r];
    MGLevel F = R.f.mg.lv[0];
    F.b = R.cg.r[a.k & 1];
    const int lb = blockIdx.x - a.off[r], tx = (F.nr + 1 + UTX - 1) / UTX;
    mg_up_cg_body(F, R.f.mg.lv[1], R.cg, a.k, lb % tx, lb / tx);
}

__global__ void __launch_bounds__(CB) k_cg_update_last_b(BatchArgs a)
{
    const int r = batch_run(a);
    const RunSolve &R = *a.run[r];
    cg_update_last_body(R.f.mg.lv[0], R.cg, a.k, blockIdx.x - a.off[r], a.off[r + 1] - a.off[r]);
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

namespace {

// Pairs (l, l + 1) of grid levels run in one two-level kernel, taken from the
// coarse end; the finest level has blocks enough to run alone.
void level_pairs(const MGHier &H, bool two_level, bool *pair)
{
    for (int l = 0; l < MAX_LEVELS; ++l) pair[l] = false;
    if (two_level)
        for (int l = H.tail.first - 2; l >= 1; l -= 2) pair[l] = true;
}

// down kernels from level `from`, the tail, up kernels back to level `to`
void launch_levels(const MGHier &H, const bool *pair, int from, int to, double *dot,
                   hipStream_t s)
{
    for (int l = from; l < H.tail.first;) {
        if (pair[l]) {
            const MGLevel &F = H.lv[l], &M = H.lv[l + 1], &C = H.lv[l + 2];
            dim3 g((C.nr + 1 + D2W - 1) / D2W, (C.nz + 1 + D2H - 1) / D2H);
            hipLaunchKernelGGL(k_mg_down2, g, dim3(D2T), 0, s, F, M, C);
            l += 2;
        } else {
            const MGLevel &F = H.lv[l], &C = H.lv[l + 1];
            dim3 g((C.nr + 1 + DTX - 1) / DTX, (C.nz + 1 + DTY - 1) / DTY);
            hipLaunchKernelGGL(k_mg_down, g, dim3(256), 0, s, F, C);
            l += 1;
        }
    }
    hipLaunchKernelGGL(k_mg_tail, dim3(1), dim3(TT, TT), H.tail_lds_bytes, s, H.tail,
                       H.tail.first == 0 ? dot : nullptr);
    for (int l = H.tail.first - 1; l >= to;) {
        if (l >= 1 && pair[l - 1] && l - 1 >= to) {
            const MGLevel &F = H.lv[l - 1], &M = H.lv[l], &C = H.lv[l + 1];
            dim3 g((F.nr + 1 + UTX - 1) / UTX, (F.nz + 1 + UTY - 1) / UTY);
            hipLaunchKernelGGL(k_mg_up2, g, dim3(256), 0, s, F, M, C);
            l -= 2;
        } else {
            const MGLevel &F = H.lv[l], &C = H.lv[l + 1];
            dim3 g((F.nr + 1 + UTX - 1) / UTX, (F.nz + 1 + UTY - 1) / UTY);
            hipLaunchKernelGGL(k_mg_up, g, dim3(256), 0, s, F, C, l == 0 ? dot : nullptr);
            l -= 1;
        }
    }
}

}  // namespace

void launch_mg_vcycle(const MGHier &H, double *dot, hipStream_t s, bool two_level)
{
    bool pair[MAX_LEVELS];
    level_pairs(H, two_level, pair);
    launch_levels(H, pair, 0, 0, dot, s);
}

void launch_mg_vcycle_cg(const MGHier &H, const CgVecs &v, int k, hipStream_t s, bool two_level)
{
    bool pair[MAX_LEVELS];
    level_pairs(H, two_level, pair);
    MGLevel F = H.lv[0];
    F.b = v.r[k & 1];
    const MGLevel &C = H.lv[1];
    dim3 gd((C.nr + 1 + DTX - 1) / DTX, (C.nz + 1 + DTY - 1) / DTY);
    if (k == 0) hipLaunchKernelGGL(k_mg_down, gd, dim3(256), 0, s, F, C);
    else hipLaunchKernelGGL(k_mg_down_cg, gd, dim3(256), 0, s, F, C, v, k - 1);
    launch_levels(H, pair, 1, 1, nullptr, s);
    dim3 gu((F.nr + 1 + UTX - 1) / UTX, (F.nz + 1 + UTY - 1) / UTY);
    hipLaunchKernelGGL(k_mg_up_cg, gu, dim3(256), 0, s, F, C, v, k);
}

void launch_cg_update_last(const MGHier &H, const CgVecs &v, int k, hipStream_t s)
{
    const MGLevel &L = H.lv[0];
    const int64_t nn = (int64_t)(L.nr + 1) * (L.nz + 1);
    hipLaunchKernelGGL(k_cg_update_last, dim3(cg_blocks(nn)), dim3(CB), 0, s, L, v, k);
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

bool batch_fused_cg(const BatchPlan &P)
{
    for (int r = 0; r < P.nruns; ++r)
        if (P.host[r].tail.first < 1) return false;
    return true;
}

// The middle levels (1 .. first - 1 of each run) one kernel per level, as in
// the unfused V-cycle; the finest level's down and up kernels carry the CG
// vector work of iterations k - 1 and k.
void launch_mg_vcycle_cg_b(const BatchPlan &P, int k, hipStream_t s)
{
    BatchArgs a = batch_args(P);
    a.k = k;
    int lmax = 0, tail_lds = 0;
    for (int r = 0; r < P.nruns; ++r) {
        lmax = std::max(lmax, (int)P.host[r].tail.first);
        tail_lds = std::max(tail_lds, (int)P.host[r].tail_lds_bytes);
    }
    for (int r = 0; r < P.nruns; ++r) {
        const MGLevel &C = P.host[r].lv[1];
        a.off[r + 1] = a.off[r] + ((C.nr + 1 + DTX - 1) / DTX) * ((C.nz + 1 + DTY - 1) / DTY);
    }
    if (k == 0) hipLaunchKernelGGL(k_mg_down_b, dim3(a.off[P.nruns]), dim3(256), 0, s, a);
    else hipLaunchKernelGGL(k_mg_down_cg_b, dim3(a.off[P.nruns]), dim3(256), 0, s, a);
    for (int l = 1; l < lmax; ++l) {
        a.level = l;
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
    for (int l = lmax - 1; l >= 1; --l) {
        a.level = l;
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
    for (int r = 0; r < P.nruns; ++r) {
        const MGLevel &F = P.host[r].lv[0];
        a.off[r + 1] = a.off[r] + ((F.nr + 1 + UTX - 1) / UTX) * ((F.nz + 1 + UTY - 1) / UTY);
    }
    hipLaunchKernelGGL(k_mg_up_cg_b, dim3(a.off[P.nruns]), dim3(256), 0, s, a);
}

void launch_cg_update_last_b(const BatchPlan &P, int k, hipStream_t s)
{
    BatchArgs a = batch_args(P);
    a.k = k;
    for (int r = 0; r < P.nruns; ++r)
        a.off[r + 1] = a.off[r] + cg_blocks((int64_t)(P.host[r].lv[0].nr + 1) * (P.host[r].lv[0].nz + 1));
    hipLaunchKernelGGL(k_cg_update_last_b, dim3(a.off[P.nruns]), dim3(CB), 0, s, a);
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
