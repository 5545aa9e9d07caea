// Plasma diagnostics (Sections 4, 5 and 7) and particle re-weighting
// (Section 5).
//
// Cell moments: every particle adds (1, v_r, v_theta, v_z, |v|^2) to its cell
// (nearest grid point, the cell it is stored in), FP64.  Particles are kept
// cell-sorted, so runs of lanes with equal cells are summed across the
// wavefront first and only the last lane of a run adds to global memory.
//
// From the moments: cell densities n = N w / V_cell, V_cell = pi (r_{i+1}^2 -
// r_i^2) dz; cell temperatures T = m (S2 / N - |S1 / N|^2) / (3 e) (cells with
// at least two particles); Debye lengths sqrt(eps0 T / (e n_e)) (Section 4
// compares the one where n_e is largest with the cell size).  Over a radial
// band of cells (Section 5: 1.0 cm < r < 1.5 cm) the axial profiles of band
// density and band potential locate the sheath edge, n_e = n_i / 2, and the
// bulk, E_z = 0 above it (Section 4), by linear interpolation between cell
// centres; the electron temperature of the sheath, pre-sheath and bulk is the
// count-weighted mean of the band cells' temperatures in each (Section 5).
#include <cmath>

#include "common.h"

namespace pic {
namespace {

constexpr double QE_D = 1.602176634e-19;
constexpr double EPS0_D = 8.8541878128e-12;
constexpr int MB = 256;     // moments kernel block
constexpr int PB = 1024;    // the one-block profile kernel

// Segmented inclusive sum over the wavefront of the five moments: lane l
// ends with the sum over lanes first..l of its run of equal keys.
__device__ __forceinline__ void run_sums(int key, double (&v)[5], int lane, bool &tail)
{
    const int prev = __shfl_up(key, 1, 64), next = __shfl_down(key, 1, 64);
    const bool head = lane == 0 || prev != key;
    tail = lane == 63 || next != key;
    const unsigned long long upto = (lane == 63) ? ~0ull : ((1ull << (lane + 1)) - 1ull);
    const int first = 63 - __clzll(__ballot(head) & upto);
    for (int o = 1; o < 64; o <<= 1) {
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            const double u = __shfl_up(v[q], o, 64);
            if (lane - o >= first) v[q] += u;
        }
    }
}

template <typename T>
__global__ void __launch_bounds__(MB) k_cell_moments(SpeciesDev<T> S, int64_t n, int nr, int nz,
                                                     double *mom)
{
    const int lane = threadIdx.x & 63;
    const int64_t ncell = (int64_t)nr * nz;
    // every thread of a block runs the same number of iterations (the
    // wavefront-wide sums need all lanes)
    for (int64_t base = (int64_t)blockIdx.x * MB; base < n; base += (int64_t)gridDim.x * MB) {
        const int64_t p = base + threadIdx.x;
        int key = -1;
        double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
        if (p < n) {
            T fr, fz;
            int i;
            key = load_pos(S, p, fr, fz, i);
            if (key >= 0) {
                const double a = (double)S.vr[p], b = (double)S.vt[p], c = (double)S.vz[p];
                v[0] = 1.0;
                v[1] = a;
                v[2] = b;
                v[3] = c;
                v[4] = a * a + b * b + c * c;
            }
        }
        bool tail;
        run_sums(key, v, lane, tail);
        if (tail && key >= 0) {
            const int i = key & 0xffff, j = key >> 16;
            if (i < nr && j < nz) {
                const int64_t cell = (int64_t)j * nr + i;
#pragma unroll
                for (int q = 0; q < 5; ++q) atomic_add_dev(&mom[q * ncell + cell], v[q]);
            }
        }
    }
}

__device__ __forceinline__ double cell_volume(int i, double dr, double dz)
{
    const double r0 = i * dr, r1 = (i + 1) * dr;
    return M_PI * (r1 * r1 - r0 * r0) * dz;
}

__device__ __forceinline__ double cell_te(double m, double n, double s1x, double s1y, double s1z,
                                          double s2)
{
    if (!(n >= 2.0)) return 0.0;
    const double mean2 = s2 / n - (s1x * s1x + s1y * s1y + s1z * s1z) / (n * n);
    return fmax(m * mean2 / (3.0 * QE_D), 0.0);
}

// Cell maps: n_e, n_i, T_e, lambda_D.
__global__ void k_plasma_maps(PlasmaDev D, PlasmaArgs A)
{
    const int64_t ncell = (int64_t)A.nr * A.nz;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < ncell;
         c += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(c % A.nr);
        const double vol = cell_volume(i, A.dr, A.dz);
        const double *me = D.mom[0];
        const double ne = me[c] * A.w[0] / vol;
        const double ni = D.mom[1][c] * A.w[1] / vol;
        const double te = cell_te(A.m_e, me[c], me[ncell + c], me[2 * ncell + c],
                                  me[3 * ncell + c], me[4 * ncell + c]);
        const double lam = (ne > 0.0 && te > 0.0) ? sqrt(EPS0_D * te / (QE_D * ne)) : INFINITY;
        D.maps[c] = ne;
        D.maps[ncell + c] = ni;
        D.maps[2 * ncell + c] = te;
        D.maps[3 * ncell + c] = lam;
    }
}

__device__ __forceinline__ double block_sum_d(double v, double *buf)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) buf[wid] = v;
    __syncthreads();
    double t = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += buf[w];
    return t;    // every thread
}

// One block: band profiles, sheath and bulk edges, region temperatures and
// the Debye length at the density peak.
__global__ void __launch_bounds__(PB) k_plasma_locate(PlasmaDev D, PlasmaArgs A, const double *phi)
{
    __shared__ double buf[PB / 64];
    __shared__ int js_min, jb_min;
    __shared__ double pk_v[PB / 64];
    __shared__ int64_t pk_c[PB / 64];
    const int nr = A.nr, nz = A.nz, ld = nr + 1;
    const int64_t ncell = (int64_t)nr * nz;
    double *ne = D.prof, *ni = D.prof + (nz + 1), *pb = D.prof + 2 * (nz + 1);
    const int nb = A.ib1 - A.ib0;
    for (int j = threadIdx.x; j <= nz; j += PB) {
        double p = 0.0;
        for (int i = A.ib0; i < A.ib1; ++i)
            p += 0.5 * (phi[(int64_t)j * ld + i] + phi[(int64_t)j * ld + i + 1]);
        pb[j] = nb > 0 ? p / nb : 0.0;
        if (j < nz) {
            double se = 0.0, si = 0.0, vol = 0.0;
            for (int i = A.ib0; i < A.ib1; ++i) {
                const int64_t c = (int64_t)j * nr + i;
                se += D.mom[0][c];
                si += D.mom[1][c];
                vol += cell_volume(i, A.dr, A.dz);
            }
            ne[j] = vol > 0.0 ? se * A.w[0] / vol : 0.0;
            ni[j] = vol > 0.0 ? si * A.w[1] / vol : 0.0;
        }
    }
    if (threadIdx.x == 0) {
        js_min = INT_MAX;
        jb_min = INT_MAX;
    }
    __syncthreads();
    // sheath edge: the first cell row with n_e >= n_i / 2
    for (int j = threadIdx.x; j < nz; j += PB)
        if (ne[j] - 0.5 * ni[j] >= 0.0) atomicMin(&js_min, j);
    __syncthreads();
    const int js = js_min;
    auto ez = [&](int j) { return -(pb[j + 1] - pb[j]) / A.dz; };
    if (js != INT_MAX)
        for (int j = max(js, 1) + (int)threadIdx.x; j < nz; j += PB)
            if (ez(j - 1) < 0.0 && ez(j) >= 0.0) atomicMin(&jb_min, j);
    __syncthreads();
    const int jb = jb_min;
    double zs = NAN, zb = NAN;
    if (js != INT_MAX) {
        if (js == 0) {
            zs = 0.0;
        } else {
            const double f0 = ne[js - 1] - 0.5 * ni[js - 1], f1 = ne[js] - 0.5 * ni[js];
            zs = (js - 0.5) * A.dz + A.dz * f0 / (f0 - f1);
        }
        if (jb != INT_MAX) {
            const double e0 = ez(jb - 1), e1 = ez(jb);
            zb = (jb - 0.5) * A.dz + A.dz * (-e0) / (e1 - e0);
        }
    }
    // region temperatures over the band cells
    double sw[3] = {0.0, 0.0, 0.0}, sn[3] = {0.0, 0.0, 0.0};
    for (int64_t k = threadIdx.x; k < (int64_t)nz * nb; k += PB) {
        const int j = (int)(k / nb), i = A.ib0 + (int)(k % nb);
        const int64_t c = (int64_t)j * nr + i;
        const double n = D.mom[0][c];
        if (!(n >= 2.0)) continue;
        const double te = D.maps[2 * ncell + c];
        const double zc = (j + 0.5) * A.dz;
        int r = 0;
        if (!isnan(zs)) {
            r = zc < zs ? 0 : 1;
            if (!isnan(zb) && zc >= zb) r = 2;
        }
        sw[r] += n * te;
        sn[r] += n;
    }
    double tw[3], tn[3];
    for (int r = 0; r < 3; ++r) {
        tw[r] = block_sum_d(sw[r], buf);
        tn[r] = block_sum_d(sn[r], buf);
    }
    // density peak (first cell of the largest n_e)
    double bv = -1.0;
    int64_t bc = 0;
    for (int64_t c = threadIdx.x; c < ncell; c += PB) {
        const double v = D.maps[c];
        if (v > bv) {
            bv = v;
            bc = c;
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        const double ov = __shfl_xor(bv, o, 64);
        const int64_t oc = __shfl_xor(bc, o, 64);
        if (ov > bv || (ov == bv && oc < bc)) {
            bv = ov;
            bc = oc;
        }
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) {
        pk_v[wid] = bv;
        pk_c[wid] = bc;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        bv = pk_v[0];
        bc = pk_c[0];
        for (int w = 1; w < PB / 64; ++w)
            if (pk_v[w] > bv || (pk_v[w] == bv && pk_c[w] < bc)) {
                bv = pk_v[w];
                bc = pk_c[w];
            }
        PlasmaOut *o = (PlasmaOut *)D.out;
        o->z_sheath = zs;
        o->z_bulk = zb;
        for (int r = 0; r < 3; ++r) {
            o->te_region[r] = tn[r] > 0.0 ? tw[r] / tn[r] : 0.0;
            o->n_region[r] = tn[r];
        }
        o->lambda_d_peak = D.maps[3 * ncell + bc];
        o->n_e_peak = D.maps[bc];
        o->te_peak = D.maps[2 * ncell + bc];
        o->peak_i = (int32_t)(bc % nr);
        o->peak_j = (int32_t)(bc / nr);
    }
}

// Re-weighting: the particles whose id is not a multiple of keep_every are
// marked absorbed (the next cell sort compacts them away).
template <typename T>
__global__ void k_reweight(SpeciesDev<T> S, int64_t n, uint32_t keep_every)
{
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * blockDim.x) {
        T fr, fz;
        int i;
        const int key = load_pos(S, p, fr, fz, i);
        if (key >= 0 && S.id[p] % keep_every != 0u)
            store_pos(S, p, false, key & 0xffff, key >> 16, fr, fz);
    }
}

}  // namespace

template <typename T>
void launch_cell_moments(const SpeciesDev<T> &S, int64_t n, int nr, int nz, double *mom,
                         hipStream_t s)
{
    if (n <= 0) return;
    const int blocks = (int)std::min<int64_t>(4096, (n + MB - 1) / MB);
    hipLaunchKernelGGL((k_cell_moments<T>), dim3(blocks), dim3(MB), 0, s, S, n, nr, nz, mom);
}

void launch_plasma(const PlasmaDev &D, const PlasmaArgs &A, const double *phi, hipStream_t s)
{
    const int64_t ncell = (int64_t)A.nr * A.nz;
    const int blocks = (int)std::min<int64_t>(2048, (ncell + 255) / 256);
    hipLaunchKernelGGL(k_plasma_maps, dim3(std::max(blocks, 1)), dim3(256), 0, s, D, A);
    hipLaunchKernelGGL(k_plasma_locate, dim3(1), dim3(PB), 0, s, D, A, phi);
}

template <typename T>
void launch_reweight(const SpeciesDev<T> &S, int64_t n, uint32_t keep_every, hipStream_t s)
{
    if (n <= 0) return;
    const int blocks = (int)std::min<int64_t>(4096, (n + 255) / 256);
    hipLaunchKernelGGL((k_reweight<T>), dim3(blocks), dim3(256), 0, s, S, n, keep_every);
}

template void launch_cell_moments<float>(const SpeciesDev<float> &, int64_t, int, int, double *,
                                         hipStream_t);
template void launch_cell_moments<double>(const SpeciesDev<double> &, int64_t, int, int, double *,
                                          hipStream_t);
template void launch_reweight<float>(const SpeciesDev<float> &, int64_t, uint32_t, hipStream_t);
template void launch_reweight<double>(const SpeciesDev<double> &, int64_t, uint32_t, hipStream_t);

}  // namespace pic
