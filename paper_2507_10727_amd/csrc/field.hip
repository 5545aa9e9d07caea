// Field kernels of libpic.so: FP64 residual and refinement of the R-Z
// charge-form operator, the FP32 geometric-multigrid preconditioner and
// conjugate-gradient pieces, the cathode circuit, the gather-field packing
// and grid diagnostics.
//
// Operator (reading of Section 3's "Gauss' law is obeyed along this axis"):
//   (K phi)_n = sum over the faces f of node n of c_f (phi_n - phi_nb),
// c_f = eps0 A_f / h_f of the clipped control volume; Dirichlet nodes are the
// anode row, the outer column and the cathode part of z = 0.  The FP32
// hierarchy stores c_f / eps0 and solves the correction equation
// K_uu e = r of the FP64 refinement, with zero correction on Dirichlet
// nodes.  Levels are vertex-centred (coarse node (I, J) = fine (2I, 2J)),
// re-discretised with the same face rule; prolongation is bilinear,
// restriction its transpose (charge is summed, so total charge is kept), the
// smoother red-black Gauss-Seidel (red-black before, black-red after, so the
// V-cycle is a symmetric preconditioner), the coarsest level a dense inverse.
#include "common.h"

namespace pic {

namespace {

constexpr int FB = 256;

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

__global__ void k_zero(uint32_t *p, int64_t words)
{
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
__global__ void __launch_bounds__(FB) k_residual64(int32_t nr, int32_t nz, const double *ce,
                                                   const double *cn, const uint8_t *kind,
                                                   const double *phi, const T *q0, const T *q1,
                                                   double *r64, DevScalars *sc)
{
    __shared__ double buf[FB / 64];
    const int ld = nr + 1;
    const int64_t nn = (int64_t)ld * (nz + 1);
    double rr = 0.0, bb = 0.0;
    for (int64_t n = (int64_t)blockIdx.x * FB + threadIdx.x; n < nn; n += (int64_t)gridDim.x * FB) {
        if (kind[n] != 0) { r64[n] = 0.0; continue; }
        const int j = (int)(n / ld), i = (int)(n - (int64_t)j * ld);
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
        if (a != 0.0) atomic_add_dev(&sc->res_rr, a);
        if (b != 0.0) atomic_add_dev(&sc->res_bb, b);
    }
}

__global__ void k_cast_scale(int64_t nn, const double *r64, double scale, float *r32, float *e32)
{
    for (int64_t n = (int64_t)blockIdx.x * FB + threadIdx.x; n < nn; n += (int64_t)gridDim.x * FB) {
        r32[n] = (float)(r64[n] * scale);
        e32[n] = 0.0f;
    }
}

__global__ void k_update64(int64_t nn, const uint8_t *kind, double *phi, const float *e32, double scale)
{
    for (int64_t n = (int64_t)blockIdx.x * FB + threadIdx.x; n < nn; n += (int64_t)gridDim.x * FB)
        if (kind[n] == 0) phi[n] += (double)e32[n] * scale;
}

// (A x)_n of a level (couplings / eps0), unknown node n.
__device__ __forceinline__ float level_ax(const Level &L, const float *x, int i, int j, int64_t n,
                                          float *diag_out)
{
    const int ld = L.nr + 1;
    float diag = 0.0f, off = 0.0f;
    if (i < L.nr) { const float c = L.ce[n]; diag += c; off += c * x[n + 1]; }
    if (i > 0) { const float c = L.ce[n - 1]; diag += c; off += c * x[n - 1]; }
    if (j < L.nz) { const float c = L.cn[n]; diag += c; off += c * x[n + ld]; }
    if (j > 0) { const float c = L.cn[n - ld]; diag += c; off += c * x[n - ld]; }
    *diag_out = diag;
    return diag * x[n] - off;
}

// First half-sweep from a zero guess: red unknowns x = b / diag, black 0.
__global__ void k_smooth_first(Level L)
{
    const int ld = L.nr + 1;
    const int64_t nn = (int64_t)ld * (L.nz + 1);
    for (int64_t n = (int64_t)blockIdx.x * FB + threadIdx.x; n < nn; n += (int64_t)gridDim.x * FB) {
        const int j = (int)(n / ld), i = (int)(n - (int64_t)j * ld);
        const float d = L.dinv[n];
        L.x[n] = (((i + j) & 1) == 0 && d != 0.0f) ? d * L.b[n] : 0.0f;
    }
}

// Gauss-Seidel update of one colour ((i + j) & 1 == color).
__global__ void k_rb(Level L, int color)
{
    const int ld = L.nr + 1;
    const int64_t nn = (int64_t)ld * (L.nz + 1);
    for (int64_t n = (int64_t)blockIdx.x * FB + threadIdx.x; n < nn; n += (int64_t)gridDim.x * FB) {
        const int j = (int)(n / ld), i = (int)(n - (int64_t)j * ld);
        if (((i + j) & 1) != color) continue;
        const float d = L.dinv[n];
        if (d == 0.0f) continue;
        float off = 0.0f;
        if (i < L.nr) off += L.ce[n] * L.x[n + 1];
        if (i > 0) off += L.ce[n - 1] * L.x[n - 1];
        if (j < L.nz) off += L.cn[n] * L.x[n + ld];
        if (j > 0) off += L.cn[n - ld] * L.x[n - ld];
        L.x[n] = d * (L.b[n] + off);
    }
}

// Coarse right-hand side = P^T (b - A x) of the fine level.
__global__ void k_restrict(Level F, Level C)
{
    const int ldc = C.nr + 1, ldf = F.nr + 1;
    const int64_t nn = (int64_t)ldc * (C.nz + 1);
    for (int64_t n = (int64_t)blockIdx.x * FB + threadIdx.x; n < nn; n += (int64_t)gridDim.x * FB) {
        const int J = (int)(n / ldc), I = (int)(n - (int64_t)J * ldc);
        float acc = 0.0f;
        if (C.dinv[n] != 0.0f) {
            for (int b = -1; b <= 1; ++b) {
                const int j = 2 * J + b;
                if (j < 0 || j > F.nz) continue;
                for (int a = -1; a <= 1; ++a) {
                    const int i = 2 * I + a;
                    if (i < 0 || i > F.nr) continue;
                    const int64_t m = (int64_t)j * ldf + i;
                    if (F.dinv[m] == 0.0f) continue;
                    float dg;
                    const float ax = level_ax(F, F.x, i, j, m, &dg);
                    const float w = (a == 0 ? 1.0f : 0.5f) * (b == 0 ? 1.0f : 0.5f);
                    acc += w * (F.b[m] - ax);
                }
            }
        }
        C.b[n] = acc;
    }
}

// Fine correction += P x_coarse (bilinear).
__global__ void k_prolong(Level C, Level F)
{
    const int ldc = C.nr + 1, ldf = F.nr + 1;
    const int64_t nn = (int64_t)ldf * (F.nz + 1);
    for (int64_t n = (int64_t)blockIdx.x * FB + threadIdx.x; n < nn; n += (int64_t)gridDim.x * FB) {
        if (F.dinv[n] == 0.0f) continue;
        const int j = (int)(n / ldf), i = (int)(n - (int64_t)j * ldf);
        const int I = i >> 1, J = j >> 1;
        const int64_t c = (int64_t)J * ldc + I;
        float v;
        if (!(i & 1) && !(j & 1)) v = C.x[c];
        else if ((i & 1) && !(j & 1)) v = 0.5f * (C.x[c] + C.x[c + 1]);
        else if (!(i & 1) && (j & 1)) v = 0.5f * (C.x[c] + C.x[c + ldc]);
        else v = 0.25f * (C.x[c] + C.x[c + 1] + C.x[c + ldc] + C.x[c + ldc + 1]);
        F.x[n] += v;
    }
}

// Coarsest level: x_u = A_uu^{-1} b_u with the dense inverse (one block).
__global__ void k_coarse_solve(Level L, const float *inv, const int32_t *map, int n)
{
    extern __shared__ float sb[];
    for (int a = threadIdx.x; a < n; a += blockDim.x) sb[a] = L.b[map[a]];
    __syncthreads();
    for (int a = threadIdx.x; a < n; a += blockDim.x) {
        float acc = 0.0f;
        const float *row = inv + (int64_t)a * n;
        for (int b = 0; b < n; ++b) acc += row[b] * sb[b];
        L.x[map[a]] = acc;
    }
}

// ---- conjugate-gradient pieces on the finest level (FP32 vectors, FP64 dots)
__global__ void __launch_bounds__(FB) k_pcg_matvec_dot(Level L, const float *p, float *q, double *pq)
{
    __shared__ double buf[FB / 64];
    const int ld = L.nr + 1;
    const int64_t nn = (int64_t)ld * (L.nz + 1);
    double acc = 0.0;
    for (int64_t n = (int64_t)blockIdx.x * FB + threadIdx.x; n < nn; n += (int64_t)gridDim.x * FB) {
        float v = 0.0f;
        if (L.dinv[n] != 0.0f) {
            const int j = (int)(n / ld), i = (int)(n - (int64_t)j * ld);
            float dg;
            v = level_ax(L, p, i, j, n, &dg);
            acc += (double)p[n] * (double)v;
        }
        q[n] = v;
    }
    const double t = block_sum(acc, buf);
    if (threadIdx.x == 0 && t != 0.0) atomic_add_dev(pq, t);
}

__global__ void __launch_bounds__(FB) k_pcg_update(int64_t nn, const double *rz, const double *pq,
                                                   const float *p, const float *q, float *e,
                                                   float *r, double *rr)
{
    __shared__ double buf[FB / 64];
    const double den = *pq;
    const float alpha = (den != 0.0) ? (float)(*rz / den) : 0.0f;
    double acc = 0.0;
    for (int64_t n = (int64_t)blockIdx.x * FB + threadIdx.x; n < nn; n += (int64_t)gridDim.x * FB) {
        e[n] += alpha * p[n];
        const float rv = r[n] - alpha * q[n];
        r[n] = rv;
        acc += (double)rv * (double)rv;
    }
    const double t = block_sum(acc, buf);
    if (threadIdx.x == 0 && t != 0.0) atomic_add_dev(rr, t);
}

__global__ void __launch_bounds__(FB) k_pcg_dot(int64_t nn, const float *a, const float *b, double *out)
{
    __shared__ double buf[FB / 64];
    double acc = 0.0;
    for (int64_t n = (int64_t)blockIdx.x * FB + threadIdx.x; n < nn; n += (int64_t)gridDim.x * FB)
        acc += (double)a[n] * (double)b[n];
    const double t = block_sum(acc, buf);
    if (threadIdx.x == 0 && t != 0.0) atomic_add_dev(out, t);
}

__global__ void k_pcg_direction(int64_t nn, const double *rz_new, const double *rz_old,
                                const float *z, float *p)
{
    const double den = *rz_old;
    const float beta = (den != 0.0) ? (float)(*rz_new / den) : 0.0f;
    for (int64_t n = (int64_t)blockIdx.x * FB + threadIdx.x; n < nn; n += (int64_t)gridDim.x * FB)
        p[n] = z[n] + beta * p[n];
}

__global__ void k_copy_f32(float *dst, const float *src, int64_t n)
{
    for (int64_t k = (int64_t)blockIdx.x * FB + threadIdx.x; k < n; k += (int64_t)gridDim.x * FB)
        dst[k] = src[k];
}

// ---- circuit: induced cathode charge of phi0 and the cathode voltage update
template <typename T>
__global__ void k_circuit(int32_t nr, const double *ce, const double *cn, const uint8_t *kind,
                          const double *phi0, const T *q0, const T *q1, DevScalars *sc,
                          int circuit, double v_fixed, double v_ext, double r_ext, double dt,
                          double extra_dq)
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

// ---- gather fields: phi = phi0 + V_c phi_L and the node 4-vectors
template <typename T>
__global__ void k_field_prep(int32_t nr, int32_t nz, double dr, double dz, double *phi,
                             const double *phi0, const double *phil, const double *br,
                             const double *bz, typename Vec4<T>::type *node, const DevScalars *sc,
                             int scheme, int use_phi)
{
    const int ld = nr + 1;
    const int64_t nn = (int64_t)ld * (nz + 1);
    const double vc = sc->vc;
    for (int64_t n = (int64_t)blockIdx.x * FB + threadIdx.x; n < nn; n += (int64_t)gridDim.x * FB) {
        const int j = (int)(n / ld), i = (int)(n - (int64_t)j * ld);
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

__global__ void k_zero_unknowns(int64_t nn, const uint8_t *kind, double *phi)
{
    for (int64_t n = (int64_t)blockIdx.x * FB + threadIdx.x; n < nn; n += (int64_t)gridDim.x * FB)
        if (kind[n] == 0) phi[n] = 0.0;
}

__global__ void k_set_dirichlet(int64_t nn, const uint8_t *kind, double *phi, double vcat)
{
    for (int64_t n = (int64_t)blockIdx.x * FB + threadIdx.x; n < nn; n += (int64_t)gridDim.x * FB) {
        if (kind[n] == 1) phi[n] = vcat;
        else if (kind[n] == 2) phi[n] = 0.0;
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
        const int j = (int)(n / ld), i = (int)(n - (int64_t)j * ld);
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

}  // namespace

void launch_zero(void *p, int64_t bytes, hipStream_t s)
{
    const int64_t words = (bytes + 3) / 4;
    hipLaunchKernelGGL(k_zero, dim3(blocks_for(words, 2048)), dim3(FB), 0, s, (uint32_t *)p, words);
}

template <typename T>
void launch_residual64(const FieldDev &f, const double *phi, const T *q0, const T *q1,
                       DevScalars *sc, hipStream_t s)
{
    const int64_t nn = (int64_t)(f.nr + 1) * (f.nz + 1);
    launch_zero(&sc->res_rr, 2 * sizeof(double), s);
    hipLaunchKernelGGL((k_residual64<T>), dim3(blocks_for(nn, 1024)), dim3(FB), 0, s, f.nr, f.nz,
                       f.ce64, f.cn64, f.kind, phi, q0, q1, f.r64, sc);
}

void launch_cast_scale(const FieldDev &f, double scale, hipStream_t s)
{
    const int64_t nn = (int64_t)(f.nr + 1) * (f.nz + 1);
    hipLaunchKernelGGL(k_cast_scale, dim3(blocks_for(nn)), dim3(FB), 0, s, nn, f.r64, scale,
                       f.r32, f.e32);
}

void launch_update64(const FieldDev &f, double *phi, double scale, hipStream_t s)
{
    const int64_t nn = (int64_t)(f.nr + 1) * (f.nz + 1);
    hipLaunchKernelGGL(k_update64, dim3(blocks_for(nn)), dim3(FB), 0, s, nn, f.kind, phi, f.e32,
                       scale);
}

static void vcycle_level(const FieldDev &f, int l, hipStream_t s)
{
    const Level &L = f.lv[l];
    const int64_t nn = (int64_t)(L.nr + 1) * (L.nz + 1);
    if (l == f.nlevels - 1) {
        hipLaunchKernelGGL(k_coarse_solve, dim3(1), dim3(256), f.coarse_n * sizeof(float), s, L,
                           f.coarse_inv, f.coarse_map, f.coarse_n);
        return;
    }
    const int nb = blocks_for(nn);
    const Level &C = f.lv[l + 1];
    const int64_t nc = (int64_t)(C.nr + 1) * (C.nz + 1);
    hipLaunchKernelGGL(k_smooth_first, dim3(nb), dim3(FB), 0, s, L);
    hipLaunchKernelGGL(k_rb, dim3(nb), dim3(FB), 0, s, L, 1);
    hipLaunchKernelGGL(k_restrict, dim3(blocks_for(nc)), dim3(FB), 0, s, L, C);
    vcycle_level(f, l + 1, s);
    hipLaunchKernelGGL(k_prolong, dim3(nb), dim3(FB), 0, s, C, L);
    hipLaunchKernelGGL(k_rb, dim3(nb), dim3(FB), 0, s, L, 1);
    hipLaunchKernelGGL(k_rb, dim3(nb), dim3(FB), 0, s, L, 0);
}

void launch_vcycle(const FieldDev &f, hipStream_t s) { vcycle_level(f, 0, s); }

void launch_pcg_matvec_dot(const FieldDev &f, DevScalars *sc, int k, hipStream_t s)
{
    const Level &L = f.lv[0];
    const int64_t nn = (int64_t)(L.nr + 1) * (L.nz + 1);
    hipLaunchKernelGGL(k_pcg_matvec_dot, dim3(blocks_for(nn, 1024)), dim3(FB), 0, s, L, f.p32,
                       f.q32, &sc->pcg_pq[k]);
}

void launch_pcg_update(const FieldDev &f, DevScalars *sc, int k, hipStream_t s)
{
    const int64_t nn = (int64_t)(f.nr + 1) * (f.nz + 1);
    hipLaunchKernelGGL(k_pcg_update, dim3(blocks_for(nn, 1024)), dim3(FB), 0, s, nn,
                       &sc->pcg_rz[k], &sc->pcg_pq[k], f.p32, f.q32, f.e32, f.r32,
                       &sc->pcg_rr[k]);
}

void launch_pcg_dot_rz(const FieldDev &f, DevScalars *sc, int k, hipStream_t s)
{
    const int64_t nn = (int64_t)(f.nr + 1) * (f.nz + 1);
    hipLaunchKernelGGL(k_pcg_dot, dim3(blocks_for(nn, 1024)), dim3(FB), 0, s, nn, f.r32, f.z32,
                       &sc->pcg_rz[k]);
}

void launch_pcg_direction(const FieldDev &f, DevScalars *sc, int k, hipStream_t s)
{
    const int64_t nn = (int64_t)(f.nr + 1) * (f.nz + 1);
    hipLaunchKernelGGL(k_pcg_direction, dim3(blocks_for(nn)), dim3(FB), 0, s, nn,
                       &sc->pcg_rz[k + 1], &sc->pcg_rz[k], f.z32, f.p32);
}

void launch_copy_f32(float *dst, const float *src, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_copy_f32, dim3(blocks_for(n)), dim3(FB), 0, s, dst, src, n);
}

template <typename T>
void launch_circuit(const FieldDev &f, const T *q0, const T *q1, DevScalars *sc, int circuit,
                    double v_fixed, double v_ext, double r_ext, double dt, double extra_dq,
                    hipStream_t s)
{
    hipLaunchKernelGGL((k_circuit<T>), dim3(1), dim3(1024), 0, s, f.nr, f.ce64, f.cn64, f.kind,
                       f.phi0, q0, q1, sc, circuit, v_fixed, v_ext, r_ext, dt, extra_dq);
}

template <typename T>
void launch_field_prep(const FieldDev &f, typename Vec4<T>::type *node, DevScalars *sc,
                       int scheme, int use_phi, hipStream_t s)
{
    const int64_t nn = (int64_t)(f.nr + 1) * (f.nz + 1);
    hipLaunchKernelGGL((k_field_prep<T>), dim3(blocks_for(nn)), dim3(FB), 0, s, f.nr, f.nz, f.dr,
                       f.dz, f.phi, f.phi0, f.phi_l, f.b_r, f.b_z, node, sc, scheme, use_phi);
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
                                       const float *, DevScalars *, hipStream_t);
template void launch_residual64<double>(const FieldDev &, const double *, const double *,
                                        const double *, DevScalars *, hipStream_t);
template void launch_circuit<float>(const FieldDev &, const float *, const float *, DevScalars *,
                                    int, double, double, double, double, double, hipStream_t);
template void launch_circuit<double>(const FieldDev &, const double *, const double *,
                                     DevScalars *, int, double, double, double, double, double,
                                     hipStream_t);
template void launch_field_prep<float>(const FieldDev &, float4 *, DevScalars *, int, int,
                                       hipStream_t);
template void launch_field_prep<double>(const FieldDev &, double4 *, DevScalars *, int, int,
                                        hipStream_t);
template void launch_diag_grid<float>(const FieldDev &, const float *, const float *, double,
                                      double, double *, int, hipStream_t);
template void launch_diag_grid<double>(const FieldDev &, const double *, const double *, double,
                                       double, double *, int, hipStream_t);

}  // namespace pic
