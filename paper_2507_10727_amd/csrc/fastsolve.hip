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
//   B     = r on the unknown block,
//   B^    = S B       (FP64 MFMA matrix product over z),
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

constexpr int GT = 32;       // C tile of a block (GT x GT), 4 waves of 16 x 16
constexpr int GK = 32;       // K slice staged in LDS per pass
constexpr int LDA_S = GK + 4;   // padded LDS row of the A slice (doubles)
constexpr int LDB_S = GT + 4;   // padded LDS row of the B slice

// C = A B for padded row-major operands: A is Mp x Kp (lda), B is Kp x Np
// (ldb); Mp, Np, Kp are multiples of 32.  Each of the 4 waves of a block
// owns one 16 x 16 quarter of the block's 32 x 32 tile and accumulates it
// with v_mfma_f64_16x16x4f64: A operand lane l = row l % 16, k = l / 16;
// B operand lane l = column l % 16, k = l / 16; result item v (0..3) of
// lane l is row l / 16 + 4 v of column l % 16 (measured on gfx950).
// Epilogue: mode 0 stores the tile to C (ldc); mode 1 adds rows m < M,
// columns n < N to the node array phi at ((m + 1) * ldp + n), the unknown
// rows 1..nz-1 of the grid.
__global__ void __launch_bounds__(256) k_gemm_f64(const double *__restrict__ A, int lda,
                                                  const double *__restrict__ B, int ldb,
                                                  double *__restrict__ C, int ldc, int Kp,
                                                  int mode, int M, int N, int ldp)
{
    __shared__ double As[2][GT * LDA_S];
    __shared__ double Bs[2][GK * LDB_S];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wm = w >> 1, wn = w & 1;
    const int m0 = blockIdx.y * GT, n0 = blockIdx.x * GT;
    // staging: each thread moves 4 doubles of A and 4 of B per slice
    // (two 16-byte loads each): A slice 32 rows x 32 k, B slice 32 k x 32 cols
    const int ar = tid >> 3, ac = (tid & 7) * 4;     // A: row, first k
    const int br = tid >> 3, bc = (tid & 7) * 4;     // B: k, first column
    const double *Ag = A + (int64_t)(m0 + ar) * lda + ac;
    const double *Bg = B + (int64_t)br * ldb + n0 + bc;
    double2 ra0 = *(const double2 *)(Ag), ra1 = *(const double2 *)(Ag + 2);
    double2 rb0 = *(const double2 *)(Bg), rb1 = *(const double2 *)(Bg + 2);
    d4 acc = {0.0, 0.0, 0.0, 0.0};
    const int nslice = Kp / GK;
    for (int s = 0; s < nslice; ++s) {
        const int buf = s & 1;
        double *as = As[buf] + ar * LDA_S + ac;
        as[0] = ra0.x; as[1] = ra0.y; as[2] = ra1.x; as[3] = ra1.y;
        double *bs = Bs[buf] + br * LDB_S + bc;
        bs[0] = rb0.x; bs[1] = rb0.y; bs[2] = rb1.x; bs[3] = rb1.y;
        __syncthreads();
        if (s + 1 < nslice) {
            const double *An = Ag + (s + 1) * GK;
            const double *Bn = Bg + (int64_t)(s + 1) * GK * ldb;
            ra0 = *(const double2 *)(An);
            ra1 = *(const double2 *)(An + 2);
            rb0 = *(const double2 *)(Bn);
            rb1 = *(const double2 *)(Bn + 2);
        }
        const double *ap = As[buf] + (wm * 16 + (lane & 15)) * LDA_S + (lane >> 4);
        const double *bp = Bs[buf] + (lane >> 4) * LDB_S + wn * 16 + (lane & 15);
#pragma unroll
        for (int kk = 0; kk < GK; kk += 4)
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(ap[kk], bp[kk * LDB_S], acc, 0, 0, 0);
        // the next pass writes the other buffer; this one is rewritten two
        // passes later, after the barrier of the next pass
    }
    const int col = n0 + wn * 16 + (lane & 15);
    const int row0 = m0 + wm * 16 + (lane >> 4);
    if (mode == 0) {
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

// Right-hand side of the correction equation on the unknown block:
// B[j-1][i] = r(i, j), the FP64 residual of the current potential, for
// i < nr, 1 <= j < nz, and zero on the rest of the padded Mp x ldb block
// (so nothing earlier left in B matters).  Also clears the residual norms'
// slots for the check that follows the correction.
__global__ void k_fs_rhs(int32_t nr, int32_t nz, const double *__restrict__ r64,
                         double *__restrict__ Bm, int ldb, int Mp, double *__restrict__ res_slots)
{
    if (blockIdx.x == 0)
        for (int k = threadIdx.x; k < RES_SLOT_WORDS; k += blockDim.x) res_slots[k] = 0.0;
    const int ld = nr + 1;
    const int64_t total = (int64_t)Mp * ldb;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int jm = (int)(t / ldb), i = (int)(t - (int64_t)jm * ldb);
        Bm[t] = (jm < nz - 1 && i < nr) ? r64[(int64_t)(jm + 1) * ld + i] : 0.0;
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
__global__ void k_solve_check(DevScalars *sc, double rtol2)
{
    if (threadIdx.x != 0) return;
    double rr = 0.0, bb = 0.0;
    for (int k = 0; k < ACC_SLOTS; ++k) {
        rr += sc->res_slots[k * ACC_STRIDE];
        bb += sc->res_slots[(ACC_SLOTS + k) * ACC_STRIDE];
    }
    if (!(rr <= rtol2 * bb)) atomicOr(&sc->flags, FLAG_NOCONV);
}

}  // namespace

void launch_solve_check(DevScalars *sc, double rtol2, hipStream_t s)
{
    hipLaunchKernelGGL(k_solve_check, dim3(1), dim3(64), 0, s, sc, rtol2);
}

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
    const int64_t total = (int64_t)Mp * Np;
    const int rb = (int)std::min<int64_t>(2048, std::max<int64_t>(1, (total + 255) / 256));
    hipLaunchKernelGGL(k_fs_rhs, dim3(rb), dim3(256), 0, s, nr, nz, (const double *)f.r64, F.b,
                       Np, Mp, sc->res_slots);
    hipLaunchKernelGGL(k_gemm_f64, dim3(Np / GT, Mp / GT), dim3(256), 0, s, F.S, Mp, F.b, Np,
                       F.bh, Np, Mp, 0, M, nr, 0);
    int pt = 64;
    while (pt < nr) pt <<= 1;
    hipLaunchKernelGGL(k_fs_pcr, dim3(M), dim3(pt), 0, s, nr, F.ce1, F.cn1, F.lam, F.bh, Np);
    hipLaunchKernelGGL(k_gemm_f64, dim3(Np / GT, Mp / GT), dim3(256), 0, s, F.S, Mp, F.bh, Np,
                       phi, 0, Mp, 1, M, nr, nr + 1);
}

}  // namespace pic
