// Direct FP64 solve of the R-Z field equation when it separates.
//
// The charge-form operator of Section 3 (Gauss's law over each node's
// control volume) couples an unknown node (i, j) to its radial neighbours
// through c_e(i) = eps0 2 pi (i + 1/2) dz and to its axial neighbours through
// c_n(i) = eps0 A_i / dz, A_i the annulus of the node.  When the cathode
// covers the whole z = 0 row (every configuration whose cathode reaches the
// outer wall), the unknowns are i = 0..nr-1, j = 1..nz-1, both couplings are
// the same on every row, and the operator is a sum of Kronecker products,
//     K = R (x) I + D (x) T,
// R tridiagonal in r (the c_e), D = diag(c_n), T = tridiag(-1, 2, -1) in z
// with Dirichlet ends.  T = S Lambda S with the orthonormal sine transform
// S_jk = sqrt(2/nz) sin(pi j k / nz) and Lambda_k = 4 sin^2(pi k / (2 nz)), so
// with Phi = S Psi every sine mode k decouples into one tridiagonal system in
// r, (R + lambda_k D) psi_k = (S B)_k.  The solve is applied to the
// correction equation K d = r of the current potential phi (r its FP64
// residual: node charge plus Dirichlet couplings minus K phi):
//   B^    = S r       (FP64 MFMA matrix product over z, r read from the
//                      node residual on the unknown block),
//   Psi   tridiagonal solve of every mode (parallel cyclic reduction in LDS),
//   phi  += S Psi     (FP64 MFMA matrix product, added into the node array).
// The rounding of the transforms is relative to the correction, not to phi,
// so a warm start (the previous step's potential) leaves a residual near
// the FP64 floor; from phi = 0 the first correction is the whole solve.
// No iteration, no atomics: the result does not depend on thread timing.
// The FP64 residual of the result is checked by the caller.
#include <algorithm>
#include <cmath>

#include "common.h"

namespace pic {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int GT = 16;       // C tile of a block (GT x GT)
constexpr int GW = 8;        // waves of a block, one k range each
constexpr int KB = 8;        // k steps (of 4) whose operands a wave loads at once

// C = S B for padded row-major operands: S is the symmetric Mp x Mp sine
// transform (lda = Mp), B is Mp x Np (ldb); Mp and Np are multiples of 32.
// A block computes one 16 x 16 tile of C with v_mfma_f64_16x16x4f64; its
// eight waves take one eighth of the k range each and their partial tiles
// are summed in LDS in wave order (no atomics: the result does not depend
// on timing).  Operands come straight from global memory (L2-resident): the
// B operand of lane l is B[k + l / 16][n0 + l % 16], and since S is
// symmetric the A operand S[m0 + l % 16][k + l / 16] is read as
// S[k + l / 16][m0 + l % 16], so both are 128-byte row segments.  A wave
// loads the operands of KB steps at a time, the next group's loads issued
// before the current group's products.  Result item v (0..3) of lane l is
// row l / 16 + 4 v of column l % 16 (measured on gfx950).
// Modes: 0 and 1 store the tile to C (ldc), 2 adds rows m < M, columns
// n < N to the node array phi at ((m + 1) * ldp + n), the unknown rows
// 1..nz-1 of the grid; mode 1 reads B as the FP64 node residual instead of a
// dense block: B[k][n] = r((k + 1) ldp + n) for k < M, n < N, else 0.
// clear (nullable): the residual norms' slots, zeroed by the first block.
__global__ void __launch_bounds__(64 * GW) k_gemm_f64(const double *__restrict__ A, int lda,
                                                      const double *__restrict__ B, int ldb,
                                                      double *__restrict__ C, int ldc, int Kp,
                                                      int mode, int M, int N, int ldp,
                                                      double *__restrict__ clear)
{
    __shared__ d4 part[GW - 1][64];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int m0 = blockIdx.y * GT, n0 = blockIdx.x * GT;
    if (clear && blockIdx.x == 0 && blockIdx.y == 0)
        for (int k = tid; k < RES_SLOT_WORDS; k += 64 * GW) clear[k] = 0.0;
    const int ks = Kp / (4 * GW);                     // k steps of a wave (>= 1)
    const int kb = w * 4 * ks + (lane >> 4);
    const int col = n0 + (lane & 15);
    const double *Ap = A + (int64_t)kb * lda + m0 + (lane & 15);
    // mode 1: B is the node residual (row k of the block = node row k + 1,
    // stride ldp), zero outside the M x N unknowns
    const bool res = mode == 1;
    const double *Bp = res ? B + (int64_t)(kb + 1) * ldp + col : B + (int64_t)kb * ldb + col;
    const int64_t bstep = res ? (int64_t)4 * ldp : (int64_t)4 * ldb;
    d4 acc = {0.0, 0.0, 0.0, 0.0};
    double a[2][KB], b[2][KB];
    auto load = [&](int g, int t0) {
#pragma unroll
        for (int t = 0; t < KB; ++t) {
            const int st = min(t0 + t, ks - 1);       // clamped: a valid address
            a[g][t] = Ap[(int64_t)(4 * st) * lda];
            if (!res) {
                b[g][t] = Bp[st * bstep];
            } else {
                const int k = kb + 4 * st;
                b[g][t] = (k < M && col < N) ? Bp[st * bstep] : 0.0;
            }
        }
    };
    auto mul = [&](int g, int t0) {
#pragma unroll
        for (int t = 0; t < KB; ++t)
            if (t0 + t < ks) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[g][t], b[g][t], acc, 0, 0, 0);
    };
    load(0, 0);
    for (int t0 = 0; t0 < ks; t0 += 2 * KB) {
        if (t0 + KB < ks) load(1, t0 + KB);
        mul(0, t0);
        if (t0 + 2 * KB < ks) load(0, t0 + 2 * KB);
        if (t0 + KB < ks) mul(1, t0 + KB);
    }
    if (w > 0) part[w - 1][lane] = acc;
    __syncthreads();
    if (w != 0) return;
#pragma unroll
    for (int q = 0; q < GW - 1; ++q) acc += part[q][lane];
    const int row0 = m0 + (lane >> 4);
    if (mode == 0 || mode == 1) {
#pragma unroll
        for (int v = 0; v < 4; ++v) C[(int64_t)(row0 + 4 * v) * ldc + col] = acc[v];
    } else {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int m = row0 + 4 * v;
            if (m < M && col < N) C[(int64_t)(m + 1) * ldp + col] += acc[v];
        }
    }
}

// Tridiagonal solve of mode k (one block per mode, one thread per radial
// node, blockDim = the power of two >= nr): (R + lambda_k D) psi = row k of
// Bh, in place.  Row i: diagonal ce(i) + ce(i-1) + lambda_k cn(i), off
// diagonals -ce(i-1) (to i-1) and -ce(i) (to i+1, absent for i = nr-1).
// Parallel cyclic reduction: log2 steps, each eliminating the neighbours at
// distance s from every equation (the matrices are diagonally dominant).
__global__ void __launch_bounds__(1024) k_fs_pcr(int32_t nr, const double *__restrict__ ce1,
                                                 const double *__restrict__ cn1,
                                                 const double *__restrict__ lam,
                                                 double *__restrict__ Bh, int ldb)
{
    __shared__ double sa[1024], sb[1024], sc[1024], sd[1024];
    const int i = threadIdx.x, n = blockDim.x;
    const int k = blockIdx.x;
    double *row = Bh + (int64_t)k * ldb;
    double a = 0.0, b = 1.0, c = 0.0, d = 0.0;
    if (i < nr) {
        const double l = lam[k];
        const double cw = (i > 0) ? ce1[i - 1] : 0.0;
        const double cE = ce1[i];
        a = -cw;
        c = (i + 1 < nr) ? -cE : 0.0;
        b = cw + cE + l * cn1[i];
        d = row[i];
    }
    for (int s = 1; s < n; s <<= 1) {
        sa[i] = a; sb[i] = b; sc[i] = c; sd[i] = d;
        __syncthreads();
        double na = 0.0, nb = b, nc = 0.0, nd = d;
        if (i - s >= 0) {
            const double k1 = a / sb[i - s];
            na = -sa[i - s] * k1;
            nb -= sc[i - s] * k1;
            nd -= sd[i - s] * k1;
        }
        if (i + s < n) {
            const double k2 = c / sb[i + s];
            nc = -sc[i + s] * k2;
            nb -= sa[i + s] * k2;
            nd -= sd[i + s] * k2;
        }
        __syncthreads();
        a = na; b = nb; c = nc; d = nd;
    }
    if (i < nr) row[i] = d / b;
}

// The residual's slotted norms of one solve, summed in slot order: flag the
// solve when ||r||^2 > rtol2 ||b||^2 (the flag stays until the host reads it).


}  // namespace

int fs_pad(int n) { return (n + 31) & ~31; }

bool fs_separable(int nr, int nz, const double *ce, const double *cn, const uint8_t *kind)
{
    const int ld = nr + 1;
    for (int j = 0; j <= nz; ++j)
        for (int i = 0; i <= nr; ++i) {
            const int expect = (j == 0 || j == nz || i == nr) ? 1 : 0;
            if ((kind[(int64_t)j * ld + i] != 0) != (expect != 0)) return false;
        }
    for (int j = 1; j < nz; ++j)
        for (int i = 0; i < nr; ++i) {
            const int64_t n = (int64_t)j * ld + i;
            if (ce[n] != ce[ld + i] || cn[n] != cn[ld + i] || cn[n - ld] != cn[ld + i]) return false;
        }
    return true;
}

void fs_tables(int nr, int nz, const double *ce, const double *cn, double *S, double *ce1,
               double *cn1, double *lam)
{
    const int M = nz - 1, Mp = fs_pad(M);
    const double pi = 3.14159265358979323846;
    const double norm = std::sqrt(2.0 / nz);
    for (int j = 0; j < Mp; ++j)
        for (int k = 0; k < Mp; ++k) {
            double v = 0.0;
            if (j < M && k < M) {
                // sin(pi (j+1)(k+1) / nz) with the argument reduced exactly
                const long long p = ((long long)(j + 1) * (k + 1)) % (2LL * nz);
                v = norm * std::sin(pi * (double)p / (double)nz);
            }
            S[(int64_t)j * Mp + k] = v;
        }
    for (int k = 0; k < Mp; ++k) {
        const double s = (k < M) ? std::sin(pi * (k + 1) / (2.0 * nz)) : 0.0;
        lam[k] = 4.0 * s * s;
    }
    const int ld = nr + 1;
    for (int i = 0; i < nr; ++i) {
        ce1[i] = ce[ld + i];
        cn1[i] = cn[ld + i];
    }
}

void launch_fast_solve(const FastSolve &F, const FieldDev &f, double *phi, DevScalars *sc,
                       hipStream_t s)
{
    const int nr = f.nr, nz = f.nz;
    const int M = nz - 1, Mp = fs_pad(M), Np = fs_pad(nr);
    // B^ = S r straight from the node residual (clears the norms' slots for
    // the check that follows the correction)
    hipLaunchKernelGGL(k_gemm_f64, dim3(Np / GT, Mp / GT), dim3(64 * GW), 0, s, F.S, Mp,
                       (const double *)f.r64, 0, F.bh, Np, Mp, 1, M, nr, nr + 1, sc->res_slots);
    int pt = 64;
    while (pt < nr) pt <<= 1;
    hipLaunchKernelGGL(k_fs_pcr, dim3(M), dim3(pt), 0, s, nr, F.ce1, F.cn1, F.lam, F.bh, Np);
    hipLaunchKernelGGL(k_gemm_f64, dim3(Np / GT, Mp / GT), dim3(64 * GW), 0, s, F.S, Mp, F.bh, Np,
                       phi, 0, Mp, 2, M, nr, nr + 1, nullptr);
}

}  // namespace pic
