// Particle kernels of libpic.so: the fused timestep kernel (field gather,
// Boris push, R-Z drift, walls, the cathode's emission queue, the
// null-collision candidate test, charge deposit), the event kernel
// (collisions, ion- and electron-induced emission, the cathode ion-energy
// record), child insertion, per-step bookkeeping and the loader.
#include <climits>

#include "common.h"

namespace pic {

// ---------------------------------------------------------------------------
// Fused particle kernel.
//
// One launch covers both species: blocks [0, nblk_e) stream the electrons,
// the rest the ions.  Each wavefront walks a contiguous range of its
// species' slots in chunks of 256; lane l owns the 4 consecutive slots
// 4l..4l+3 of a chunk and moves them with one 16-byte load and store per
// array, so a wavefront reads and writes 1 KiB contiguous segments.
// Particles are kept sorted by cell, so a lane's 4 particles usually share
// a cell: the 4 node 4-vectors of the gather are loaded once per distinct
// cell, and the deposit is summed in registers per run of equal cells, then
// per run of equal cells across lanes, before it goes to LDS.  Each
// wavefront accumulates its charge in a window of node rows held in its own
// LDS tile, kept from chunk to chunk while its (sorted) particles stay
// inside, and adds a window to the global charge with one atomic per
// nonzero node when it moves on; a chunk too spread for a window uses global
// atomics.  The wavefronts of a block never wait for each other, so one's
// loads overlap another's deposit.
//
// Per particle (Section 2 for the gather, Section 3 for walls, emission and
// collisions):
//   E from the node 4-vectors: EC-PIC takes E_r from the two r-edges of the
//     cell (NGP in r, linear in z) and E_z from the two z-edges (linear in r,
//     NGP in z); MC-PIC interpolates nodal E with the deposit's tent weights;
//     B is tent-interpolated in both.
//   Boris rotation in the Cartesian frame (r-hat, theta-hat, z-hat) at the
//     particle, drift, and rotation of (v_r, v_theta) into the new
//     meridional plane; the radial displacement is formed as
//     (2 r dx + dx^2 + dy^2) / (r + r') so that the cell-relative position
//     keeps full precision in FP32.
//   Walls in priority z < 0 (cathode if r < cathode_rmax, else the Neumann
//     block), r >= R, z >= L; an absorbed slot is marked (key -1, or pz = -1
//     in the packed FP32 state).
//   Collisions for surviving electrons that existed before the step.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void iso_direction(uint32_t ua, uint32_t ub, T &d0, T &d1, T &d2)
{
    const T c = (T)1 - (T)2 * u24<T>(ua);
    // sin(chi) from (1 - c)(1 + c): both factors are exact for c = 1 - 2U,
    // where 1 - c^2 would cancel near c = +-1
    const T s = sqrt(fmax((T)0, ((T)1 - c) * ((T)1 + c)));
    T sn, cs;
    sincos_2pi(u24<T>(ub), &sn, &cs);
    d0 = s * cs;
    d1 = s * sn;
    d2 = c;
}

template <typename T>
__device__ __forceinline__ void record_child(const PushCold<T> *C, DevScalars *sc,
                                             int parent_species, uint32_t parent_id, int kind,
                                             int species, int i, int j, T fr, T fz, T vr, T vt,
                                             T vz)
{
    const int slot = atomicAdd(&sc->n_child, 1);
    atomicAdd(&sc->n_child_s[species], 1);
    if (slot >= C->child_cap) {
        atomicOr(&sc->flags, FLAG_CHILD_OVERFLOW);
        return;
    }
    Child<T> c;
    c.skey = ((unsigned long long)parent_species << 33) | ((unsigned long long)parent_id << 1) |
             (unsigned long long)kind;
    c.species = species;
    c.key = (j << 16) | i;
    c.fr = fr;
    c.fz = fz;
    c.vr = vr;
    c.vt = vt;
    c.vz = vz;
    C->child[slot] = c;
}

template <typename T>
__device__ __forceinline__ T interp_row(const T *row, int k, T f)
{
    return ((T)1 - f) * row[k] + f * row[k + 1];
}

template <typename T> __device__ __forceinline__ T near_one();
template <> __device__ __forceinline__ float near_one<float>() { return 0x1.fffffep-1f; }
template <> __device__ __forceinline__ double near_one<double>() { return 0x1.fffffffffffffp-1; }

// Reciprocal and square root: the hardware approximations (about 1 ulp) in
// FP32, exact operations in FP64 (the FP64 state is compared with the oracle
// at 1e-12).
template <typename T> __device__ __forceinline__ T rcp(T x);
template <> __device__ __forceinline__ float rcp<float>(float x) { return __builtin_amdgcn_rcpf(x); }
template <> __device__ __forceinline__ double rcp<double>(double x) { return 1.0 / x; }
template <typename T> __device__ __forceinline__ T fast_sqrt(T x);
template <> __device__ __forceinline__ float fast_sqrt<float>(float x) { return __builtin_amdgcn_sqrtf(x); }
template <> __device__ __forceinline__ double fast_sqrt<double>(double x) { return sqrt(x); }

struct Tally {
    double ke = 0.0, pz = 0.0;
    unsigned int abs1 = 0, abs2 = 0, abs3 = 0, abs4 = 0;
    unsigned int cand = 0, el = 0, ex = 0, iz = 0, see = 0, fb = 0;
};

// Gather, Boris, drift and walls for one particle.  Updates the state in
// place and returns 0 if it stays inside, else the wall code (1 cathode,
// 2 Neumann block, 3 outer r, 4 anode).  ke_dot / pz_v receive
// v^{n-1/2}.v^{n+1/2} and v_z^{n+1/2} for the diagnostics.
template <typename T, int SCHEME>
__device__ __forceinline__ int advance(const PushParams<T> &P, T hqm, uint32_t dbits,
                                       const typename Vec4<T>::type &a00,
                                       const typename Vec4<T>::type &a10,
                                       const typename Vec4<T>::type &a01,
                                       const typename Vec4<T>::type &a11, int &i, int &j, T &fr,
                                       T &fz, T &vr, T &vt, T &vz, T &ke_dot, T &pz_v)
{
    // Every rounding is written out (fused multiply-adds explicit, no
    // contraction left to the compiler): the kernel handles up to four
    // particles per thread in unrolled copies of this code, and a particle's
    // result must not depend on which copy it falls in.
#pragma clang fp contract(off)
    const int nr = P.nr, nz = P.nz;
    const T gr = (T)1 - fr, gz = (T)1 - fz;
    const T w00 = gr * gz, w10 = fr * gz, w01 = gr * fz, w11 = fr * fz;
    auto tent = [&](T c00, T c10, T c01, T c11) {
        return fma(w00, c00, fma(w10, c10, fma(w01, c01, w11 * c11)));
    };
    T er, ez;
    if (SCHEME == PIC_EC) {
        er = fma(gz, a00.x, fz * a01.x);
        ez = fma(gr, a00.y, fr * a10.y);
    } else {
        er = tent(a00.x, a10.x, a01.x, a11.x);
        ez = tent(a00.y, a10.y, a01.y, a11.y);
    }
    const T br = tent(a00.z, a10.z, a01.z, a11.z);
    const T bz = tent(a00.w, a10.w, a01.w, a11.w);
    // Boris: half kick, rotation about t = (q dt / 2m) B, half kick
    const T mx = fma(hqm, er, vr), my = vt, mz = fma(hqm, ez, vz);
    const T tx = hqm * br, tz = hqm * bz;
    const T f2 = (T)2 * rcp<T>(fma(tx, tx, fma(tz, tz, (T)1)));
    const T sx = f2 * tx, sz = f2 * tz;
    const T px = fma(my, tz, mx);
    const T py = my + fma(mz, tx, -(mx * tz));
    const T pzz = fma(-my, tx, mz);
    const T qx = fma(py, sz, mx);
    const T qy = my + fma(pzz, sx, -(px * sz));
    const T qz = fma(-py, sx, mz);
    const T nx = fma(hqm, er, qx), ny = qy, nzv = fma(hqm, ez, qz);
    ke_dot = fma(vr, nx, fma(vt, ny, vz * nzv));
    pz_v = nzv;
    // drift in (x, y, z) = (r, 0, z), rotate into the new meridional plane
    const T r = ((T)i + fr) * P.dr;
    const T dx = nx * P.dt, dy = ny * P.dt;
    const T x1 = r + dx;
    const T r1 = fast_sqrt(fma(x1, x1, dy * dy));
    T vr1 = nx, vt1 = ny, vz1 = nzv;
    if (r1 > (T)0) {
        const T inv = rcp<T>(r1);
        const T c = x1 * inv, sn = dy * inv;
        vr1 = fma(c, nx, sn * ny);
        vt1 = fma(c, ny, -(sn * nx));
    }
    const T den = r + r1;
    const T drr = (den > (T)0) ? fma((T)2 * r, dx, fma(dx, dx, dy * dy)) * rcp<T>(den) : (T)0;
    T xr, xz;
    if constexpr (sizeof(T) == 4) {
        // displacements rounded to the state's quanta without bias (dbits:
        // 16 dither bits per axis), so the new offsets are exact
        xr = fr + step_round(drr * P.inv_dr, dbits & 0xFFFFu);
        xz = fz + step_round((nzv * P.dt) * P.inv_dz, dbits >> 16);
    } else {
        xr = fma(drr, P.inv_dr, fr);
        xz = fma(nzv * P.dt, P.inv_dz, fz);
    }
    const T flr = floor(xr), flz = floor(xz);
    int i1 = i + (int)flr, j1 = j + (int)flz;
    T fr1 = xr - flr, fz1 = xz - flz;
    if (fr1 >= (T)1) { fr1 = (T)0; ++i1; }
    if (fz1 >= (T)1) { fz1 = (T)0; ++j1; }
    int fate = 0;
    if (!P.any_reflect) {
        if (j1 < 0) fate = (r1 < P.cold->cathode_rmax) ? 1 : 2;
        else if (i1 >= nr) fate = 3;
        else if (j1 >= nz) fate = 4;
    } else {
        const int *wbc = P.cold->wall_bc;
        if (j1 < 0) {
            if (wbc[0] == PIC_REFLECT) {
                const T zg = -((T)j1 + fz1);
                const T fl = floor(zg);
                j1 = (int)fl;
                fz1 = zg - fl;
                if (fz1 >= (T)1) { fz1 = (T)0; ++j1; }
                vz1 = -vz1;
            } else {
                fate = (r1 < P.cold->cathode_rmax) ? 1 : 2;
            }
        }
        if (fate == 0 && i1 >= nr) {
            if (wbc[2] == PIC_REFLECT) {
                const T rg = (T)(2 * nr) - ((T)i1 + fr1);
                const T fl = floor(rg);
                i1 = (int)fl;
                fr1 = rg - fl;
                if (i1 >= nr) { i1 = nr - 1; fr1 = near_one<T>(); }
                vr1 = -vr1;
            } else {
                fate = 3;
            }
        }
        if (fate == 0 && j1 >= nz) {
            if (wbc[1] == PIC_REFLECT) {
                const T zg = (T)(2 * nz) - ((T)j1 + fz1);
                const T fl = floor(zg);
                j1 = (int)fl;
                fz1 = zg - fl;
                if (j1 >= nz) { j1 = nz - 1; fz1 = near_one<T>(); }
                vz1 = -vz1;
            } else {
                fate = 4;
            }
        }
    }
    if (fate == 0) {
        // r' >= 0 exactly; round-off can put i' at -1 next to the axis.  Any
        // index still outside the grid (non-finite or absurd velocities under
        // reflecting walls) is clamped so every access stays in bounds.
        if (i1 < 0) { i1 = 0; fr1 = (T)0; }
        if (i1 > nr - 1) { i1 = nr - 1; fr1 = near_one<T>(); }
        if (j1 < 0) { j1 = 0; fz1 = (T)0; }
        if (j1 > nz - 1) { j1 = nz - 1; fz1 = near_one<T>(); }
        if (!(fr1 >= (T)0 && fr1 < (T)1)) fr1 = (T)0;
        if (!(fz1 >= (T)0 && fz1 < (T)1)) fz1 = (T)0;
    }
    i = i1;
    j = j1;
    fr = fr1;
    fz = fz1;
    vr = vr1;
    vt = vt1;
    vz = vz1;
    return fate;
}

// Ionization products of one collision (from the ground state or from the
// metastable: `threshold` is 15.76 or 4.20 eV).  Returns the scattered
// electron's energy; records the ejected electron and the new ion as
// children.
template <typename T>
__device__ __forceinline__ T ionize(const PushCold<T> *C, DevScalars *sc, uint32_t id,
                                 uint32_t word1, uint32_t step, uint32_t key0, uint32_t key1,
                                 int i, int j, T fr, T fz, T e, T threshold)
{
    const T erem = e - threshold;
    const uint4 ua = philox4x32_10(make_uint4(id, word1 | PURPOSE_IZ, step, 0u), key0, key1);
    const uint4 ub = philox4x32_10(make_uint4(id, word1 | PURPOSE_ION, step, 0u), key0, key1);
    const T eej = u24<T>(ua.x) * erem;
    T e0, e1, e2;
    iso_direction(ua.y, ua.z, e0, e1, e2);
    const T vej = sqrt(C->v2_of_e * eej);
    record_child(C, sc, 0, id, 0, 0, i, j, fr, fz, vej * e0, vej * e1, vej * e2);
    const T a0 = sqrt((T)-2 * log(u_open<T>(ub.x)));
    const T a1 = sqrt((T)-2 * log(u_open<T>(ub.z)));
    T s0, c0, s1, cb;
    sincos_2pi(u24<T>(ub.y), &s0, &c0);
    sincos_2pi(u24<T>(ub.w), &s1, &cb);
    const T sg = C->sig_ion;
    record_child(C, sc, 0, id, 1, 1, i, j, fr, fz, sg * a0 * c0, sg * a0 * s0, sg * a1 * cb);
    return ((T)1 - u24<T>(ua.x)) * erem;   // = erem - eej, without cancellation
}

// The selected collision of one candidate electron: energy, process, new
// velocity, ionization products.
template <typename T>
__device__ __forceinline__ void scatter(const PushCold<T> *C, DevScalars *sc, uint4 u, uint32_t id,
                                     uint32_t word1, uint32_t step, uint32_t key0, uint32_t key1,
                                     int i, int j, T fr, T fz, T *v, unsigned int *counts)
{
    T vr = v[0], vt = v[1], vz = v[2];
    const int nt = C->n_table;
    const T v2 = vr * vr + vt * vt + vz * vz;
    const T e = C->e_of_v2 * v2;
    const T x = e * C->inv_de;
    int kk;
    T f;
    if (x >= (T)(nt - 1)) { kk = nt - 2; f = (T)1; }
    else { const T fl = floor(x); kk = (int)fl; f = x - fl; }
    const T c1 = interp_row(C->nu, kk, f);
    const T c2 = c1 + interp_row(C->nu + nt, kk, f);
    const T c3 = c2 + interp_row(C->nu + 2 * nt, kk, f);
    const T c4 = c3 + interp_row(C->nu + 3 * nt, kk, f);
    const T rsel = u24<T>(u.y) * C->numax;
    int proc = -1;
    if (rsel < c1) proc = 0;
    else if (rsel < c2) proc = (e >= C->e_exc) ? 1 : -1;
    else if (rsel < c3) proc = (e >= C->e_iz) ? 2 : -1;
    else if (rsel < c4) proc = (e >= C->e_iz_meta) ? 3 : -1;
    if (proc < 0) return;
    counts[proc]++;
    T d0, d1, d2;
    iso_direction(u.z, u.w, d0, d1, d2);
    T enew;
    if (proc == 0) {
        const T vm = sqrt(v2);
        const T cth = (vr * d0 + vt * d1 + vz * d2) / vm;
        enew = e * ((T)1 - C->two_m_over_M * ((T)1 - cth));
    } else if (proc == 1) {
        enew = e - C->e_exc;
    } else {
        enew = ionize(C, sc, id, word1, step, key0, key1, i, j, fr, fz, e,
                      proc == 2 ? C->e_iz : C->e_iz_meta);
    }
    const T vn = sqrt(C->v2_of_e * enew);
    v[0] = vn * d0;
    v[1] = vn * d1;
    v[2] = vn * d2;
}

// Lane moves of the data-parallel primitives (DPP): row_shr:n shifts by n
// lanes within rows of 16, row_bcast:15 / :31 pass lane 15 of a row (lane 31)
// to the next row (to the upper half).  Lanes without a source read 0.
template <int CTRL, int ROWS>
__device__ __forceinline__ float dpp_move(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROWS, 0xF, true));
}
template <int CTRL, int ROWS>
__device__ __forceinline__ long long dpp_move(long long b)
{
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, ROWS, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROWS, 0xF, true);
    return ((long long)hi << 32) | (long long)(unsigned)lo;
}
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_move(double v)
{
    return __longlong_as_double(dpp_move<CTRL, ROWS>(__double_as_longlong(v)));
}

// Segmented inclusive sum over the wavefront: lane l ends with the sum of
// lanes first..l of its segment (first = the segment's first lane), computed
// with four in-row shifts and two row broadcasts.
template <typename T>
__device__ __forceinline__ void wave_segment_sum(T &a0, T &a1, T &a2, T &a3, int lane, int first)
{
#define PIC_SEG_STEP(CTRL, ROWS, COND)                                                  \
    {                                                                                 \
        const T b0 = dpp_move<CTRL, ROWS>(a0), b1 = dpp_move<CTRL, ROWS>(a1);         \
        const T b2 = dpp_move<CTRL, ROWS>(a2), b3 = dpp_move<CTRL, ROWS>(a3);         \
        if (COND) {                                                                   \
            a0 += b0;                                                                 \
            a1 += b1;                                                                 \
            a2 += b2;                                                                 \
            a3 += b3;                                                                 \
        }                                                                             \
    }
    PIC_SEG_STEP(0x111, 0xF, (lane & 15) >= 1 && lane - 1 >= first)
    PIC_SEG_STEP(0x112, 0xF, (lane & 15) >= 2 && lane - 2 >= first)
    PIC_SEG_STEP(0x114, 0xF, (lane & 15) >= 4 && lane - 4 >= first)
    PIC_SEG_STEP(0x118, 0xF, (lane & 15) >= 8 && lane - 8 >= first)
    PIC_SEG_STEP(0x142, 0xA, ((lane >> 4) & 1) && first <= (lane & ~15) - 1)
    PIC_SEG_STEP(0x143, 0xC, lane >= 32 && first <= 31)
#undef PIC_SEG_STEP
}

// How the deposit accumulates.  Floating: tent weights summed in T, scaled
// by q w when added to a node.  Fixed point (FP64 state): each particle's
// weights rounded to 64-bit fixed point and summed as integers, so the sums
// do not depend on the order of the additions; q w is applied when the node
// charge is converted after the step's last deposit.  The wavefront's tile
// is addressed through LDS pointers, so its atomics are LDS instructions.
template <typename A>
using lds_ptr = __attribute__((address_space(3))) A *;

template <typename T, bool FIXED>
struct DepAcc {
    using A = T;
    static __device__ __forceinline__ A weight(T w) { return w; }
    static __device__ __forceinline__ A scaled(A a, T qw) { return qw * a; }
    static __device__ __forceinline__ void dev_add(A *p, A v) { atomic_add_dev(p, v); }
};
template <typename T>
struct DepAcc<T, true> {
    using A = long long;
    static __device__ __forceinline__ A weight(T w) { return to_fixed((double)w); }
    static __device__ __forceinline__ A scaled(A a, T) { return a; }
    static __device__ __forceinline__ void dev_add(A *p, A v)
    {
        atomicAdd((unsigned long long *)p, (unsigned long long)v);
    }
};

template <typename A>
__device__ __forceinline__ void lds_add(lds_ptr<A> p, A v)
{
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}

// Add one run's summed tent weights to its cell's four nodes: in the
// wavefront's LDS tile (key relative to the tile) or in global memory.
template <typename D, typename T>
__device__ __forceinline__ void deposit_lds(lds_ptr<typename D::A> tile, int ld, int key, T qw,
                                            typename D::A a00, typename D::A a10,
                                            typename D::A a01, typename D::A a11)
{
    const int i = key & 0xffff, j = key >> 16;
    lds_ptr<typename D::A> p = tile + (j * ld + i);
    lds_add(p, D::scaled(a00, qw));
    lds_add(p + 1, D::scaled(a10, qw));
    lds_add(p + ld, D::scaled(a01, qw));
    lds_add(p + ld + 1, D::scaled(a11, qw));
}
template <typename D, typename T>
__device__ __forceinline__ void deposit_dev(typename D::A *q, int ld, int key, T qw,
                                            typename D::A a00, typename D::A a10,
                                            typename D::A a01, typename D::A a11)
{
    const int i = key & 0xffff, j = key >> 16;
    typename D::A *p = q + ((int64_t)j * ld + i);
    D::dev_add(p, D::scaled(a00, qw));
    D::dev_add(p + 1, D::scaled(a10, qw));
    D::dev_add(p + ld, D::scaled(a01, qw));
    D::dev_add(p + ld + 1, D::scaled(a11, qw));
}

// Wavefront-wide minimum / maximum, uniform in every lane: lane moves
// within rows of 16 (DPP: swap neighbours, swap pairs, mirror halves,
// mirror the row), then the four row results read from lanes 15, 31, 47, 63.
template <bool MAX>
__device__ __forceinline__ int wave_extreme(int v)
{
    auto op = [](int a, int b) { return MAX ? max(a, b) : min(a, b); };
    v = op(v, __builtin_amdgcn_update_dpp(v, v, 0xB1, 0xF, 0xF, false));
    v = op(v, __builtin_amdgcn_update_dpp(v, v, 0x4E, 0xF, 0xF, false));
    v = op(v, __builtin_amdgcn_update_dpp(v, v, 0x141, 0xF, 0xF, false));
    v = op(v, __builtin_amdgcn_update_dpp(v, v, 0x140, 0xF, 0xF, false));
    const int a = __builtin_amdgcn_readlane(v, 15), b = __builtin_amdgcn_readlane(v, 31);
    const int c = __builtin_amdgcn_readlane(v, 47), d = __builtin_amdgcn_readlane(v, 63);
    return op(op(a, b), op(c, d));
}

// The wavefront's deposit window: node rows [j0, j0 + h) x columns
// [i0, i0 + w) of the grid held in its LDS tile (h w <= the tile's nodes).
// A wavefront walks a contiguous range of cell-sorted particles, so its
// chunks mostly fall in one window; the window is written to global memory
// (one atomic per nonzero node) only when a chunk leaves it and at the end.
struct DepWindow {
    int i0, j0, w, h;
    bool on;
};

// Add the window's nonzero nodes to the global charge and clear them.
template <typename D>
__device__ __forceinline__ void window_flush(lds_ptr<typename D::A> tile, DepWindow &win,
                                             typename D::A *Q, int ldn, int lane)
{
    using A = typename D::A;
    if (!win.on) return;
    wave_sync();
    for (int r = 0; r < win.h; ++r) {
        const lds_ptr<A> row = tile + r * win.w;
        A *const qrow = Q + (int64_t)(win.j0 + r) * ldn + win.i0;
        for (int c = lane; c < win.w; c += 64) {
            const A v = row[c];
            if (v != (A)0) {
                D::dev_add(qrow + c, v);
                row[c] = (A)0;
            }
        }
    }
    wave_sync();
    win.on = false;
}

// Deposit of the wavefront's chunk (up to four particles a lane; ok[k] is
// the cell key of particle k, -1 for none) into its window; a chunk outside
// the window moves it (flush, then a window around the chunk's node
// bounding box), and a chunk too spread for any window goes straight to
// global memory.  Every lane of the wavefront takes part.
template <typename T, bool FIXED, int WAVE_NODES>
__device__ __forceinline__ void deposit_chunk(const int (&ok)[4], const T (&fr)[4],
                                              const T (&fz)[4], lds_ptr<T> tile_mem, void *q_mem,
                                              int ldn, T qw, int lane, unsigned int &fb,
                                              DepWindow &win)
{
    using D = DepAcc<T, FIXED>;
    using A = typename D::A;
    static_assert(sizeof(A) == sizeof(T), "the tile holds T-sized words");
    const lds_ptr<A> tile = (lds_ptr<A>)tile_mem;
    A *const Q = (A *)q_mem;
    bool fits = win.on;
    if (fits) {
        bool mine = true;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (ok[k] < 0) continue;
            const int i = ok[k] & 0xffff, j = ok[k] >> 16;
            mine = mine && (unsigned)(i - win.i0) < (unsigned)(win.w - 1) &&
                   (unsigned)(j - win.j0) < (unsigned)(win.h - 1);
        }
        fits = __ballot(!mine) == 0ull;
    }
    if (!fits) {
        int imin = INT_MAX, imax = INT_MIN, jmin = INT_MAX, jmax = INT_MIN;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (ok[k] < 0) continue;
            const int i = ok[k] & 0xffff, j = ok[k] >> 16;
            imin = min(imin, i); imax = max(imax, i);
            jmin = min(jmin, j); jmax = max(jmax, j);
        }
        imin = wave_extreme<false>(imin); imax = wave_extreme<true>(imax);
        jmin = wave_extreme<false>(jmin); jmax = wave_extreme<true>(jmax);
        if (imax < imin) return;                 // no particle in the chunk
        window_flush<D>(tile, win, Q, ldn, lane);
        // three node rows (a cell row and its neighbours' drift), as many
        // columns as the tile holds from one column before the chunk (the
        // wavefront's later chunks lie at larger keys)
        const int h = max(jmax - jmin + 2, 3);
        const int i0 = max(imin - 1, 0);
        const int w = min(WAVE_NODES / h, ldn - i0);
        if (imax + 2 - i0 <= w) {
            win.i0 = i0;
            win.j0 = jmin;
            win.w = w;
            win.h = h;
            win.on = true;
        } else if (lane == 0) {
            ++fb;
        }
    }
    const int shift = (win.j0 << 16) | win.i0;
    const bool use_lds = win.on;
    auto add_run = [&](int key, A a00, A a10, A a01, A a11) {
        if (use_lds) deposit_lds<D>(tile, win.w, key - shift, qw, a00, a10, a01, a11);
        else deposit_dev<D>(Q, ldn, key, qw, a00, a10, a01, a11);
    };
    // the thread's particles summed per run of equal cells: the first run
    // joins the wavefront's per-cell sum, later runs (the thread's particles
    // span a cell boundary) are added directly
    int cur = -1, key0 = -1;
    A s00 = 0, s10 = 0, s01 = 0, s11 = 0;
    A f00 = 0, f10 = 0, f01 = 0, f11 = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (ok[k] < 0) continue;
        if (ok[k] != cur) {
            if (cur >= 0) {
                if (key0 < 0) {
                    key0 = cur;
                    f00 = s00; f10 = s10; f01 = s01; f11 = s11;
                } else {
                    add_run(cur, s00, s10, s01, s11);
                }
            }
            cur = ok[k];
            s00 = s10 = s01 = s11 = (A)0;
        }
        const T gr = (T)1 - fr[k], gz = (T)1 - fz[k];
        s00 += D::weight(gr * gz);
        s10 += D::weight(fr[k] * gz);
        s01 += D::weight(gr * fz[k]);
        s11 += D::weight(fr[k] * fz[k]);
    }
    if (cur >= 0) {
        if (key0 < 0) {
            key0 = cur;
            f00 = s00; f10 = s10; f01 = s01; f11 = s11;
        } else {
            add_run(cur, s00, s10, s01, s11);
        }
    }
    // per-cell sums over the wavefront's lanes: adjacent lanes whose first
    // runs share a cell form a segment, its last lane adds the total (sorted
    // particles make segments long, so few lanes add and the LDS atomics
    // rarely meet on one address)
    const bool valid = key0 >= 0;
    // neighbours' keys by whole-wavefront lane shifts (DPP wave_shr / wave_shl
    // by one; the end lanes keep their own key and are decided by lane index)
    const int prev = __builtin_amdgcn_update_dpp(key0, key0, 0x138, 0xF, 0xF, false);
    const int next = __builtin_amdgcn_update_dpp(key0, key0, 0x130, 0xF, 0xF, false);
    const bool head = valid && (lane == 0 || prev != key0);
    const bool tail = valid && (lane == 63 || next != key0);
    const unsigned long long upto = (lane == 63) ? ~0ull : ((1ull << (lane + 1)) - 1ull);
    const unsigned long long hb = __ballot(head) & upto;
    const int first = hb ? 63 - __clzll(hb) : lane;
    wave_segment_sum(f00, f10, f01, f11, lane, first);
    if (tail) add_run(key0, f00, f10, f01, f11);
}

// Append (slot, aux) to an event queue.  Entries past the capacity are
// dropped and flagged.
__device__ __forceinline__ void enqueue(int2 *q, int *count, int cap, int slot, int aux)
{
    const int e = atomicAdd(count, 1);
    if (e < cap) q[e] = make_int2(slot, aux);
}

// Impact point of an ion absorbed on the cathode, carried by its emission
// queue entry: FP32 state passes the packed radial word (the slot keeps no
// position once absorbed), FP64 state the radial cell, the offset staying in
// the slot.
template <typename T>
__device__ __forceinline__ int see_aux(int i, T fr)
{
    if constexpr (sizeof(T) == 4) return (int)pos_pack(min(max(i, 0), POS_MAX_CELLS - 1), fr);
    else return i;
}
template <typename T>
__device__ __forceinline__ void see_impact(const SpeciesDev<T> &S, int2 q, int &i, T &fr)
{
    if constexpr (sizeof(T) == 4) {
        i = pos_cell((uint32_t)q.y);
        fr = pos_frac((uint32_t)q.y);
    } else {
        i = q.y;
        fr = S.fr[q.x];
    }
}

// Streaming 16-byte loads and stores of the particle arrays.  The arrays
// pass through once per step, so they are marked non-temporal: they do not
// displace the node arrays of the gather from the caches.
template <typename V, typename E>
__device__ __forceinline__ V stream_load_v(const V *p)
{
    typedef E vec __attribute__((ext_vector_type(4)));
    const vec t = __builtin_nontemporal_load((const vec *)p);
    V r;
    r.x = t[0];
    r.y = t[1];
    r.z = t[2];
    r.w = t[3];
    return r;
}
template <typename V, typename E>
__device__ __forceinline__ void stream_store_v(V *p, const V &v)
{
    typedef E vec __attribute__((ext_vector_type(4)));
    const vec t = {v.x, v.y, v.z, v.w};
    __builtin_nontemporal_store(t, (vec *)p);
}
__device__ __forceinline__ int4 stream_load(const int4 *p) { return stream_load_v<int4, int>(p); }
__device__ __forceinline__ uint4 stream_load(const uint4 *p) { return stream_load_v<uint4, unsigned>(p); }
__device__ __forceinline__ float4 stream_load(const float4 *p) { return stream_load_v<float4, float>(p); }
__device__ __forceinline__ double4 stream_load(const double4 *p) { return stream_load_v<double4, double>(p); }
__device__ __forceinline__ void stream_store(int4 *p, const int4 &v) { stream_store_v<int4, int>(p, v); }
__device__ __forceinline__ void stream_store(float4 *p, const float4 &v) { stream_store_v<float4, float>(p, v); }
__device__ __forceinline__ void stream_store(double4 *p, const double4 &v) { stream_store_v<double4, double>(p, v); }

// Marks the four words of a loaded vector as used here.  Every word of a
// chunk's loads is then waited for at one point on every path through the
// loop body; a word left unread on some path (a masked-off particle, a frozen
// species) would otherwise make the compiler wait for all memory operations
// at the loop's back edge, the stores just issued included.
template <typename V>
__device__ __forceinline__ void consume(const V &v)
{
    asm volatile("" ::"v"(v.x), "v"(v.y), "v"(v.z), "v"(v.w));
}

// The particle kernel's work for block bid of the nb blocks given to one
// run, of which the first nblk_e push electrons and the rest ions.
template <typename T, int SCHEME>
__device__ __forceinline__ void push_body(const PushParams<T> P, int bid, int nb, int nblk_e)
{
    using T4 = typename Vec4<T>::type;
    constexpr int NW = PUSH_THREADS / 64;
    constexpr int WAVE_NODES = LDS_NODES / NW;
    __shared__ T lds_q[LDS_NODES];
    __shared__ double dred[2][NW];
    __shared__ unsigned long long cred[10][NW];

    const int tid = threadIdx.x;
    const int lane = tid & 63, wid = tid >> 6;
    const lds_ptr<T> tile = (lds_ptr<T>)(lds_q + wid * WAVE_NODES);
    const int s = (bid < nblk_e) ? 0 : 1;
    const int blk = s ? bid - nblk_e : bid;
    const int nblk = s ? nb - nblk_e : nblk_e;
    int32_t *__restrict__ KEY = P.sp[s].key;
    T *__restrict__ FR = P.sp[s].fr;
    T *__restrict__ FZ = P.sp[s].fz;
    T *__restrict__ VR = P.sp[s].vr;
    T *__restrict__ VT = P.sp[s].vt;
    T *__restrict__ VZ = P.sp[s].vz;
    const uint32_t *__restrict__ ID = P.sp[s].id;
    const T4 *__restrict__ NODE = P.node;
    const int64_t n = P.sc->count[s];
    const uint32_t step = (uint32_t)P.sc->step;
    const int ldn = P.nr + 1;
    const T hqm = P.hqm[s], qw = P.qw[s];
    const bool frozen = P.deposit_only || ((s == 1) && P.frozen_ions);
    const bool collide_on = (s == 0) && P.mcc_on && !P.deposit_only;
    const bool emit = P.emit[s] != 0;
    const uint32_t word1 = (P.run << 8) | ((uint32_t)s << 4);
    T *__restrict__ Q = P.q[s];
    Tally t;

    // Each wavefront takes a contiguous range of the species' chunks of 64 x
    // PUSH_PPT particles.  The particles are cell-sorted, so the range covers
    // a compact run of cells (its deposit stays in one LDS window), and
    // wavefronts running at the same time work on distant cells (their
    // global charge atomics do not meet on the same nodes).
    constexpr int WCHUNK = 64 * PUSH_PPT;
    const int64_t nch = (n + WCHUNK - 1) / WCHUNK;
    const int64_t wv = (int64_t)blk * NW + wid, nwv = (int64_t)nblk * NW;
    const int64_t c_end = (wv + 1) * nch / nwv;
    DepWindow win = {0, 0, 0, 0, false};
    for (int q = lane; q < WAVE_NODES; q += 64) tile[q] = (T)0;
    // FP32: the deposit of a chunk runs in the next iteration, between the
    // issue of that chunk's loads and their first use, so it overlaps their
    // latency (FP64 deposits in place: the held words would cost occupancy)
    int pok[4] = {-1, -1, -1, -1};
    T pfr[4] = {(T)0, (T)0, (T)0, (T)0}, pfz[4] = {(T)0, (T)0, (T)0, (T)0};
    auto deposit_prev = [&]() {
        if constexpr (sizeof(T) == 8) {
            if (P.fixed_q)
                deposit_chunk<T, true, WAVE_NODES>(pok, pfr, pfz, tile, Q, ldn, qw, lane, t.fb, win);
            else
                deposit_chunk<T, false, WAVE_NODES>(pok, pfr, pfz, tile, Q, ldn, qw, lane, t.fb, win);
        } else {
            deposit_chunk<T, false, WAVE_NODES>(pok, pfr, pfz, tile, Q, ldn, qw, lane, t.fb, win);
        }
    };
    // Null-collision candidates of a chunk take one range of the event queue
    // for the whole wavefront, reserved by one atomic (the ballots of the four
    // particle positions rank the entries); the entries are written in the
    // next iteration, once that chunk's loads are issued, so the end of an
    // iteration holds only the particle stores.
    unsigned int pend = 0;          // bit k: particle k of the lane's held chunk
    uint32_t prank = 0;             // byte k: entry of particle k within the range
    int pend_base = 0, pleader = -1;
    int64_t pp0 = 0;
    auto flush_mcc = [&]() {
        if (pleader < 0) return;
        const int base = __builtin_amdgcn_readlane(pend_base, pleader);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int e = base + (int)((prank >> (8 * k)) & 0xFFu);
            if ((pend & (1u << k)) && e < P.ev_cap) P.mcc_q[e] = make_int2((int)(pp0 + k), 0);
        }
        pleader = -1;
        pend = 0;
    };
    for (int64_t c = wv * nch / nwv; c < c_end; ++c) {
        const int64_t p0 = c * WCHUNK + 4 * lane;
        int kk[4];
        T fr[4], fz[4], vr[4], vt[4], vz[4];
        uint32_t id[4] = {0u, 0u, 0u, 0u};
        // slots p0..p0+3 are inside the (4-rounded) capacity; those at or
        // beyond the count are masked and written back unchanged; a lane past
        // the end reads slot 0 and discards it.  Every load of the chunk is
        // issued before any of them is used, so the wavefront waits for
        // memory once per chunk.
        const bool any = p0 < n;
        const int64_t pl = any ? p0 : 0;
        if constexpr (sizeof(T) == 4) {
            const uint4 wr = stream_load((const uint4 *)(FR + pl));
            const int4 wz = stream_load((const int4 *)(FZ + pl));
            const T4 c4 = stream_load((const T4 *)(VR + pl));
            const T4 d = stream_load((const T4 *)(VT + pl));
            const T4 e = stream_load((const T4 *)(VZ + pl));
            uint4 iv = make_uint4(0u, 0u, 0u, 0u);
            if (collide_on) iv = stream_load((const uint4 *)(ID + pl));
            deposit_prev();
            consume(wr);
            consume(wz);
            consume(c4);
            consume(d);
            consume(e);
            consume(iv);
            const uint32_t r4[4] = {wr.x, wr.y, wr.z, wr.w};
            const int32_t z4[4] = {wz.x, wz.y, wz.z, wz.w};
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                // branch-free: an absorbed slot (pz = -1) gives key -1, fz 0
                const uint32_t zc = (uint32_t)max(z4[k], 0);
                fr[k] = pos_frac(r4[k]);
                fz[k] = pos_frac(zc);
                kk[k] = ((pos_cell(zc) << 16) | pos_cell(r4[k])) | (z4[k] >> 31);
            }
            vr[0] = c4.x; vr[1] = c4.y; vr[2] = c4.z; vr[3] = c4.w;
            vt[0] = d.x; vt[1] = d.y; vt[2] = d.z; vt[3] = d.w;
            vz[0] = e.x; vz[1] = e.y; vz[2] = e.z; vz[3] = e.w;
            id[0] = iv.x; id[1] = iv.y; id[2] = iv.z; id[3] = iv.w;
        } else {
            const int4 k4 = stream_load((const int4 *)(KEY + pl));
            const T4 a = stream_load((const T4 *)(FR + pl));
            const T4 b = stream_load((const T4 *)(FZ + pl));
            const T4 c4 = stream_load((const T4 *)(VR + pl));
            const T4 d = stream_load((const T4 *)(VT + pl));
            const T4 e = stream_load((const T4 *)(VZ + pl));
            uint4 iv = make_uint4(0u, 0u, 0u, 0u);
            if (collide_on) iv = stream_load((const uint4 *)(ID + pl));
            consume(k4);
            consume(a);
            consume(b);
            consume(c4);
            consume(d);
            consume(e);
            consume(iv);
            kk[0] = k4.x; kk[1] = k4.y; kk[2] = k4.z; kk[3] = k4.w;
            fr[0] = a.x; fr[1] = a.y; fr[2] = a.z; fr[3] = a.w;
            fz[0] = b.x; fz[1] = b.y; fz[2] = b.z; fz[3] = b.w;
            vr[0] = c4.x; vr[1] = c4.y; vr[2] = c4.z; vr[3] = c4.w;
            vt[0] = d.x; vt[1] = d.y; vt[2] = d.z; vt[3] = d.w;
            vz[0] = e.x; vz[1] = e.y; vz[2] = e.z; vz[3] = e.w;
            id[0] = iv.x; id[1] = iv.y; id[2] = iv.z; id[3] = iv.w;
        }
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (p0 + k >= n) kk[k] = -1;
        flush_mcc();
        unsigned int cmask = 0;
        int ok[4];   // cell key after the push, -1 if none
        T ke_c = (T)0, pz_c = (T)0;
        if (!frozen) {
            int prev = -2;
            T4 a00, a10, a01, a11;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                ok[k] = -1;
                const int key = kk[k];
                if (key < 0) continue;
                int i = key & 0xffff, j = key >> 16;
                if (key != prev) {
                    const T4 *nb = NODE + (int64_t)j * ldn + i;
                    a00 = nb[0];
                    a10 = nb[1];
                    a01 = nb[ldn];
                    a11 = nb[ldn + 1];
                    prev = key;
                }
                T kd, pv;
                const uint32_t db = (sizeof(T) == 4) ? dither_bits((uint32_t)(p0 + k), step, word1) : 0u;
                const int fate = advance<T, SCHEME>(P, hqm, db, a00, a10, a01, a11, i, j, fr[k],
                                                    fz[k], vr[k], vt[k], vz[k], kd, pv);
                ke_c += kd;
                pz_c += pv;
                if (fate) {
                    kk[k] = -1;
                    if (fate == 1) {
                        ++t.abs1;
                        // emission is decided in the event kernel; the
                        // entry's slot carries the species in bit 31
                        if (emit || (s == 1 && P.ied_on))
                            enqueue(P.see_q, &P.sc->n_see_q, P.ev_cap,
                                    (int)((uint32_t)(p0 + k) | ((uint32_t)s << 31)),
                                    see_aux<T>(i, fr[k]));
                    } else if (fate == 2) {
                        ++t.abs2;
                    } else if (fate == 3) {
                        ++t.abs3;
                    } else {
                        ++t.abs4;
                    }
                    continue;
                }
                if (collide_on) {
                    // null-collision candidate test; the collision itself is
                    // done in the event kernel for the few candidates
                    const uint4 u = philox4x32_10(make_uint4(id[k], word1 | PURPOSE_MCC, step, 0u),
                                                  P.key0, P.key1);
                    if ((unsigned long long)u.x < P.t_null) cmask |= 1u << k;
                }
                fr[k] = pos_round(fr[k]);   // the stored (FP32: rounded) offsets
                fz[k] = pos_round(fz[k]);
                kk[k] = ok[k] = (j << 16) | i;
            }
            if (collide_on) {
                // entry of particle k: candidates at positions < k in all
                // lanes, then those at position k in lower lanes (at most
                // 255 before the last of 256)
                int tot = 0;
                uint64_t any_m = 0ull;
                uint32_t rank = 0;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const uint64_t m = __ballot((cmask >> k) & 1u);
                    const uint32_t r = (uint32_t)tot + __builtin_amdgcn_mbcnt_hi(
                                                           (uint32_t)(m >> 32),
                                                           __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
                    rank |= (r & 0xFFu) << (8 * k);
                    tot += __popcll(m);
                    any_m |= m;
                }
                if (tot) {
                    const int leader = __ffsll((long long)any_m) - 1;
                    int b = 0;
                    if (lane == leader) b = atomicAdd(&P.sc->n_mcc_q, tot);
                    pend_base = b;
                    pleader = leader;
                    prank = rank;
                    pend = cmask;
                    pp0 = p0;
                }
            }
            if (any) {
                if constexpr (sizeof(T) == 4) {
                    uint32_t r4[4];
                    int32_t z4[4];
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        // an absorbed slot keeps no position (pz = -1, pr = 0)
                        r4[k] = kk[k] >= 0 ? pos_pack(kk[k] & 0xffff, fr[k]) : 0u;
                        z4[k] = kk[k] >= 0 ? (int32_t)pos_pack(kk[k] >> 16, fz[k]) : -1;
                    }
                    stream_store((int4 *)(FR + p0), make_int4((int)r4[0], (int)r4[1], (int)r4[2], (int)r4[3]));
                    stream_store((int4 *)(FZ + p0), make_int4(z4[0], z4[1], z4[2], z4[3]));
                } else {
                    stream_store((int4 *)(KEY + p0), make_int4(kk[0], kk[1], kk[2], kk[3]));
                    T4 a, b;
                    a.x = fr[0]; a.y = fr[1]; a.z = fr[2]; a.w = fr[3];
                    b.x = fz[0]; b.y = fz[1]; b.z = fz[2]; b.w = fz[3];
                    stream_store((T4 *)(FR + p0), a);
                    stream_store((T4 *)(FZ + p0), b);
                }
                T4 c, d, e;
                c.x = vr[0]; c.y = vr[1]; c.z = vr[2]; c.w = vr[3];
                d.x = vt[0]; d.y = vt[1]; d.z = vt[2]; d.w = vt[3];
                e.x = vz[0]; e.y = vz[1]; e.z = vz[2]; e.w = vz[3];
                stream_store((T4 *)(VR + p0), c);
                stream_store((T4 *)(VT + p0), d);
                stream_store((T4 *)(VZ + p0), e);
            }
        } else {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                ok[k] = kk[k];
                if (kk[k] >= 0 && !P.deposit_only) {
                    ke_c += vr[k] * vr[k] + vt[k] * vt[k] + vz[k] * vz[k];
                    pz_c += vz[k];
                }
            }
        }
        // per-chunk diagnostics in FP32, summed over chunks in FP64
        t.ke += (double)ke_c;
        t.pz += (double)pz_c;

        // ---- deposit of the chunk: FP32 in the next iteration (or after the
        // loop), FP64 here
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            pok[k] = ok[k];
            pfr[k] = fr[k];
            pfz[k] = fz[k];
        }
        if constexpr (sizeof(T) == 8) deposit_prev();
    }
    flush_mcc();
    if constexpr (sizeof(T) == 4) deposit_prev();
    if constexpr (sizeof(T) == 8) {
        if (P.fixed_q)
            window_flush<DepAcc<T, true>>((lds_ptr<long long>)tile, win, (long long *)Q, ldn, lane);
        else
            window_flush<DepAcc<T, false>>(tile, win, Q, ldn, lane);
    } else {
        window_flush<DepAcc<T, false>>(tile, win, Q, ldn, lane);
    }

    // ---- block totals of the diagnostics, one atomic per quantity
    const double mw = P.mw[s];
    double dv[2] = {wave_sum(0.5 * mw * t.ke), wave_sum(mw * t.pz)};
    unsigned long long c[10] = {t.abs1, t.abs2, t.abs3, t.abs4, 0, 0, 0, 0, 0, t.fb};
#pragma unroll
    for (int q = 0; q < 10; ++q) c[q] = wave_sum_u64(c[q]);
    if (lane == 0) {
        for (int q = 0; q < 2; ++q) dred[q][wid] = dv[q];
        for (int q = 0; q < 10; ++q) cred[q][wid] = c[q];
    }
    __syncthreads();
    if (tid == 0) {
        double a = 0, b = 0;
        unsigned long long tt[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
        for (int w = 0; w < NW; ++w) {
            a += dred[0][w];
            b += dred[1][w];
            for (int q = 0; q < 10; ++q) tt[q] += cred[q][w];
        }
        DevScalars *sc = P.sc;
        if (a != 0.0) atomic_add_dev(&sc->ke[s], a);
        if (b != 0.0) atomic_add_dev(&sc->pz[s], b);
        for (int q = 0; q < 4; ++q)
            if (tt[q]) atomicAdd(&sc->n_abs[s][q + 1], tt[q]);
        if (tt[4]) atomicAdd(&sc->n_cand, tt[4]);
        for (int q = 0; q < 3; ++q)
            if (tt[5 + q]) atomicAdd(&sc->n_coll[q], tt[5 + q]);
        if (tt[8]) atomicAdd(&sc->n_see, tt[8]);
        if (tt[9]) atomicAdd(&sc->deposit_fallback, tt[9]);
    }
}

template <typename T, int SCHEME>
__global__ void __launch_bounds__(PUSH_THREADS) k_push(PushParams<T> P)
{
    push_body<T, SCHEME>(P, (int)blockIdx.x, (int)gridDim.x, P.nblk_e);
}

// Run of block b in a batched launch: the last run whose first block is at
// most b.
template <typename T>
__device__ inline int batch_run(const PartBatch<T> &B, int b)
{
    int lo = 0, hi = B.nruns - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (B.off[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// The particle kernel of every run of an ensemble in one launch: a block
// finds its run from the block offsets and reads the run's parameters from
// the run's descriptor in device memory.
template <typename T, int SCHEME>
__global__ void __launch_bounds__(PUSH_THREADS) k_push_b(PartBatch<T> B)
{
    const int b = (int)blockIdx.x;
    const int r = batch_run(B, b);
    push_body<T, SCHEME>(B.p[r]->push, b - B.off[r], B.off[r + 1] - B.off[r], B.aux[r]);
}

// ---------------------------------------------------------------------------
// Events of the step: collisions of the null-collision candidates (queue of
// electron slots) and secondary emission of the ions absorbed on the cathode
// (queue of ion slots with their radial cell).  Each outcome depends only on
// the particle's id, the step and its state after the push, so processing
// order does not matter.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void events_body(const EventParams<T> &P, int bid, int nb)
{
    const PushCold<T> *C = P.cold;
    DevScalars *sc = P.sc;
    const uint32_t step = (uint32_t)sc->step;
    const int nm = min(sc->n_mcc_q, P.ev_cap);
    const int ns = min(sc->n_see_q, P.ev_cap);
    unsigned int coll[4] = {0u, 0u, 0u, 0u}, see[2] = {0u, 0u};
    const uint32_t w_e = P.run << 8;
    for (int e = bid * blockDim.x + threadIdx.x; e < nm + ns; e += nb * blockDim.x) {
        if (e < nm) {
            const int p = P.mcc_q[e].x;
            const SpeciesDev<T> S = P.sp[0];
            T pfr, pfz;
            int pi;
            const int key = load_pos(S, p, pfr, pfz, pi);
            const uint32_t id = S.id[p];
            const uint4 u = philox4x32_10(make_uint4(id, w_e | PURPOSE_MCC, step, 0u), P.key0, P.key1);
            T v[3] = {S.vr[p], S.vt[p], S.vz[p]};
            scatter(C, sc, u, id, w_e, step, P.key0, P.key1, key & 0xffff, key >> 16, pfr, pfz, v,
                    coll);
            S.vr[p] = v[0];
            S.vt[p] = v[1];
            S.vz[p] = v[2];
        } else {
            // an absorbed cathode hit of either species (bit 31 of the slot)
            int2 q = P.see_q[e - nm];
            const int s = (int)((uint32_t)q.x >> 31);
            q.x = (int)((uint32_t)q.x & 0x7fffffffu);
            const uint32_t pid = P.sp[s].id[q.x];
            if (s == 1 && P.ied_hist) {
                // energy record of the ion at the cathode (Section 7)
                int ie;
                T fe;
                see_impact(P.sp[1], q, ie, fe);
                const double r = ((double)ie + (double)fe) * P.dr;
                if (r >= P.ied_r0 && r < P.ied_r1) {
                    const double a = (double)P.sp[1].vr[q.x], b = (double)P.sp[1].vt[q.x];
                    const double c = (double)P.sp[1].vz[q.x];
                    const double e_ev = 0.5 * P.ied_m * (a * a + b * b + c * c) / 1.602176634e-19;
                    const double x = floor(e_ev / P.ied_emax * P.ied_nbins);
                    const int bin = (x >= (double)P.ied_nbins) ? P.ied_nbins : (int)x;
                    atomicAdd(&P.ied_hist[bin], 1ull);
                }
            }
            const uint32_t word = (P.run << 8) | ((uint32_t)s << 4) | PURPOSE_SEE;
            const uint4 u = philox4x32_10(make_uint4(pid, word, step, 0u), P.key0, P.key1);
            if ((unsigned long long)u.x < C->t_see[s]) {
                ++see[s];
                int ie;
                T fe;
                see_impact(P.sp[s], q, ie, fe);
                if (ie > P.nr - 1) { ie = P.nr - 1; fe = near_one<T>(); }
                if (ie < 0) { ie = 0; fe = (T)0; }
                record_child(C, sc, s, pid, 0, 0, ie, 0, fe, (T)0, (T)0, (T)0, (T)0);
            }
        }
    }
    for (int q = 0; q < 4; ++q)
        if (coll[q]) atomicAdd(&sc->n_coll[q], (unsigned long long)coll[q]);
    if (see[1]) atomicAdd(&sc->n_see, (unsigned long long)see[1]);
    if (see[0]) atomicAdd(&sc->n_see_e, (unsigned long long)see[0]);
    if (bid == 0 && threadIdx.x == 0) {
        sc->n_cand = (unsigned long long)nm;
        if (sc->n_mcc_q > P.ev_cap || sc->n_see_q > P.ev_cap) atomicOr(&sc->flags, FLAG_CHILD_OVERFLOW);
    }
}

template <typename T>
__global__ void __launch_bounds__(256) k_events(EventParams<T> P)
{
    events_body<T>(P, (int)blockIdx.x, (int)gridDim.x);
}

template <typename T>
__global__ void __launch_bounds__(256) k_events_b(PartBatch<T> B)
{
    const int b = (int)blockIdx.x;
    const int r = batch_run(B, b);
    events_body<T>(B.p[r]->ev, b - B.off[r], B.off[r + 1] - B.off[r]);
}

template <typename T>
void launch_events(const EventParams<T> &p, hipStream_t s)
{
    hipLaunchKernelGGL((k_events<T>), dim3(256), dim3(256), 0, s, p);
}

template <typename T>
void launch_events_b(const PartBatch<T> &b, hipStream_t s)
{
    hipLaunchKernelGGL((k_events_b<T>), dim3(b.off[b.nruns]), dim3(256), 0, s, b);
}

template <typename T>
void launch_push_b(const PartBatch<T> &b, int scheme, hipStream_t s)
{
    if (scheme == PIC_EC)
        hipLaunchKernelGGL((k_push_b<T, PIC_EC>), dim3(b.off[b.nruns]), dim3(PUSH_THREADS), 0, s, b);
    else
        hipLaunchKernelGGL((k_push_b<T, PIC_MC>), dim3(b.off[b.nruns]), dim3(PUSH_THREADS), 0, s, b);
}

template <typename T>
void launch_push(const PushParams<T> &p, int scheme, int nblocks, hipStream_t s)
{
    if (scheme == PIC_EC)
        hipLaunchKernelGGL((k_push<T, PIC_EC>), dim3(nblocks), dim3(PUSH_THREADS), 0, s, p);
    else
        hipLaunchKernelGGL((k_push<T, PIC_MC>), dim3(nblocks), dim3(PUSH_THREADS), 0, s, p);
}

// ---------------------------------------------------------------------------
// Children: ids and slots in (parent species, parent id, kind) order.
// The rank of a child among the children of its species is the number of
// such children with a smaller ordering key (keys are unique), counted over
// LDS-staged tiles of the child list.  Its slot is count[s] + rank and its id
// next_id[s] + rank; its charge is deposited with global atomics.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void children_body(const ChildParams<T> &P, int bid, int nb, unsigned long long *tk,
                              int *ts)
{
    const int n = min(P.sc->n_child, P.child_cap);
    const int ldn = P.nr + 1;
    for (int base = bid * 256; base < n; base += nb * 256) {
        const int c = base + threadIdx.x;
        unsigned long long my = ~0ull;
        int ms = -1;
        if (c < n) {
            my = P.child[c].skey;
            ms = P.child[c].species;
        }
        int rank = 0;
        for (int t0 = 0; t0 < n; t0 += 256) {
            __syncthreads();
            const int t = t0 + threadIdx.x;
            tk[threadIdx.x] = (t < n) ? P.child[t].skey : ~0ull;
            ts[threadIdx.x] = (t < n) ? P.child[t].species : -2;
            __syncthreads();
            const int lim = min(256, n - t0);
            for (int q = 0; q < lim; ++q) rank += (ts[q] == ms && tk[q] < my) ? 1 : 0;
        }
        if (c < n) {
            const Child<T> ch = P.child[c];
            const int s = ch.species;
            const int64_t slot = P.sc->count[s] + rank;
            if (slot >= P.cap[s]) {
                atomicOr(&P.sc->flags, FLAG_CAPACITY);
            } else {
                const SpeciesDev<T> S = P.sp[s];
                const int i = ch.key & 0xffff, j = ch.key >> 16;
                const T fr = pos_round(ch.fr), fz = pos_round(ch.fz);
                store_pos(S, slot, true, i, j, fr, fz);
                S.vr[slot] = ch.vr;
                S.vt[slot] = ch.vt;
                S.vz[slot] = ch.vz;
                S.id[slot] = P.sc->next_id[s] + (uint32_t)rank;
                const int64_t n0 = (int64_t)j * ldn + i;
                const T qw = P.qw[s], gr = (T)1 - fr, gz = (T)1 - fz;
                bool fixed = false;
                if constexpr (sizeof(T) == 8) fixed = P.fixed_q != 0;
                if (fixed) {
                    using D = DepAcc<T, true>;
                    long long *q = (long long *)P.q[s];
                    D::dev_add(q + n0, D::weight(gr * gz));
                    D::dev_add(q + n0 + 1, D::weight(fr * gz));
                    D::dev_add(q + n0 + ldn, D::weight(gr * fz));
                    D::dev_add(q + n0 + ldn + 1, D::weight(fr * fz));
                } else {
                    atomic_add_dev(&P.q[s][n0], qw * gr * gz);
                    atomic_add_dev(&P.q[s][n0 + 1], qw * fr * gz);
                    atomic_add_dev(&P.q[s][n0 + ldn], qw * gr * fz);
                    atomic_add_dev(&P.q[s][n0 + ldn + 1], qw * fr * fz);
                }
            }
        }
    }
}

template <typename T>
__global__ void __launch_bounds__(256) k_children(ChildParams<T> P)
{
    __shared__ unsigned long long tk[256];
    __shared__ int ts[256];
    children_body<T>(P, (int)blockIdx.x, (int)gridDim.x, tk, ts);
}

template <typename T>
__global__ void __launch_bounds__(256) k_children_b(PartBatch<T> B)
{
    __shared__ unsigned long long tk[256];
    __shared__ int ts[256];
    const int b = (int)blockIdx.x;
    const int r = batch_run(B, b);
    children_body<T>(B.p[r]->ch, b - B.off[r], B.off[r + 1] - B.off[r], tk, ts);
}

template <typename T>
void launch_children(const ChildParams<T> &p, hipStream_t s)
{
    int blocks = (p.child_cap + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL((k_children<T>), dim3(blocks), dim3(256), 0, s, p);
}

int children_b_blocks(int32_t child_cap)
{
    return std::max(1, std::min(64, (child_cap + 255) / 256));
}

template <typename T>
void launch_children_b(const PartBatch<T> &b, hipStream_t s)
{
    hipLaunchKernelGGL((k_children_b<T>), dim3(b.off[b.nruns]), dim3(256), 0, s, b);
}

// Counts and id counters advance by the children of the step; the step
// counter advances.  The charge into the cathode is formed from the step's
// integer tallies (particles of each species absorbed there, electrons
// emitted from it), which makes it independent of the order of events.
__device__ void finalize_body(DevScalars *sc, int64_t cap0, int64_t cap1, double qw_e,
                              double qw_i)
{
    const int64_t cap[2] = {cap0, cap1};
    sc->dq_conv = (double)sc->n_abs[0][1] * qw_e + (double)sc->n_abs[1][1] * qw_i -
                  (double)(sc->n_see + sc->n_see_e) * qw_e;
    for (int s = 0; s < 2; ++s) {
        int64_t c = sc->count[s] + sc->n_child_s[s];
        if (c > cap[s]) c = cap[s];
        sc->count[s] = c;
        sc->next_id[s] += (uint32_t)sc->n_child_s[s];
    }
    sc->n_child = 0;
    sc->n_child_s[0] = 0;
    sc->n_child_s[1] = 0;
    sc->n_mcc_q = 0;
    sc->n_see_q = 0;
    sc->step += 1;
}

__global__ void k_finalize_step(DevScalars *sc, int64_t cap0, int64_t cap1, double qw_e,
                                double qw_i)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    finalize_body(sc, cap0, cap1, qw_e, qw_i);
}

// one thread per run
template <typename T>
__global__ void k_finalize_b(PartBatch<T> B)
{
    const int r = (int)threadIdx.x;
    if (r >= B.nruns) return;
    const ChildParams<T> &C = B.p[r]->ch;
    finalize_body(C.sc, C.cap[0], C.cap[1], C.qw64[0], C.qw64[1]);
}

void launch_finalize_step(DevScalars *sc, const int64_t cap[2], const double qw64[2],
                          hipStream_t s)
{
    hipLaunchKernelGGL(k_finalize_step, dim3(1), dim3(64), 0, s, sc, cap[0], cap[1], qw64[0],
                       qw64[1]);
}

// Node charge of both species from fixed point (in place): the integer sum
// of rounded tent weights times q w 2^-42.  Exact conversion below 2^53,
// then one rounding of the product.
__global__ void k_q_from_fixed(long long *q0, long long *q1, int64_t nodes, double s0, double s1)
{
    for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < nodes;
         n += (int64_t)gridDim.x * blockDim.x) {
        const long long a = q0[n], b = q1[n];
        ((double *)q0)[n] = (double)a * s0;
        ((double *)q1)[n] = (double)b * s1;
    }
}

void launch_q_from_fixed(void *q0, void *q1, int64_t nodes, const double qw64[2], hipStream_t s)
{
    const double u = ldexp(1.0, -QFIX_BITS);
    const int blocks = (int)std::min<int64_t>(1024, (nodes + 255) / 256);
    hipLaunchKernelGGL(k_q_from_fixed, dim3(std::max(blocks, 1)), dim3(256), 0, s,
                       (long long *)q0, (long long *)q1, nodes, qw64[0] * u, qw64[1] * u);
}

template <typename T>
void launch_finalize_b(const PartBatch<T> &b, hipStream_t s)
{
    hipLaunchKernelGGL((k_finalize_b<T>), dim3(1), dim3(MAX_BATCH), 0, s, b);
}

// Zero the deposit targets and the per-step tallies.
__device__ void begin_body(DevScalars *sc, uint32_t *q0, uint32_t *q1, int64_t words, int bid,
                           int nb)
{
    for (int64_t k = (int64_t)bid * blockDim.x + threadIdx.x; k < words;
         k += (int64_t)nb * blockDim.x) {
        q0[k] = 0u;
        q1[k] = 0u;
    }
    if (bid == 0 && threadIdx.x == 0) {
        sc->dq_conv = 0.0;
        sc->ke[0] = sc->ke[1] = 0.0;
        sc->pz[0] = sc->pz[1] = 0.0;
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 5; ++b) sc->n_abs[a][b] = 0;
        sc->n_cand = 0;
        sc->n_coll[0] = sc->n_coll[1] = sc->n_coll[2] = sc->n_coll[3] = 0;
        sc->n_see = 0;
        sc->n_see_e = 0;
        sc->deposit_fallback = 0;
    }
}

__global__ void k_begin_step(DevScalars *sc, uint32_t *q0, uint32_t *q1, int64_t words)
{
    begin_body(sc, q0, q1, words, (int)blockIdx.x, (int)gridDim.x);
}

template <typename T>
__global__ void __launch_bounds__(256) k_begin_b(PartBatch<T> B)
{
    const int b = (int)blockIdx.x;
    const int r = batch_run(B, b);
    const PushParams<T> &P = B.p[r]->push;
    const int64_t words = (int64_t)(P.nr + 1) * (P.nz + 1) * (int64_t)(sizeof(T) / 4);
    begin_body(P.sc, (uint32_t *)P.q[0], (uint32_t *)P.q[1], words, b - B.off[r],
               B.off[r + 1] - B.off[r]);
}

int begin_b_blocks(int64_t nodes, int elem_bytes)
{
    const int64_t words = nodes * elem_bytes / 4;
    return (int)std::max<int64_t>(1, std::min<int64_t>(512, (words + 255) / 256));
}

template <typename T>
void launch_begin_b(const PartBatch<T> &b, hipStream_t s)
{
    hipLaunchKernelGGL((k_begin_b<T>), dim3(b.off[b.nruns]), dim3(256), 0, s, b);
}

void launch_begin_step(DevScalars *sc, void *q0, void *q1, int64_t nodes, int elem_bytes,
                       hipStream_t s)
{
    const int64_t words = nodes * elem_bytes / 4;
    int blocks = (int)((words + 255) / 256);
    if (blocks > 2048) blocks = 2048;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_begin_step, dim3(blocks), dim3(256), 0, s, sc, (uint32_t *)q0,
                       (uint32_t *)q1, words);
}

// Loader: absolute FP64 positions -> cell and in-cell fraction (stored as
// the state's layout has it), i = floor(r / dr) kept in [0, nr-1],
// fr = r/dr - i.
template <typename T>
__global__ void k_load(SpeciesDev<T> S, int64_t off, const double *r, const double *z,
                       const double *vr, const double *vt, const double *vz, const uint32_t *id,
                       int64_t n, int32_t nr, int32_t nz, double dr, double dz)
{
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n;
         k += (int64_t)gridDim.x * blockDim.x) {
        const double x = r[k] / dr, y = z[k] / dz;
        int i = (int)floor(x), j = (int)floor(y);
        i = max(0, min(nr - 1, i));
        j = max(0, min(nz - 1, j));
        T fr = (T)(x - i), fz = (T)(y - j);
        if (fr >= (T)1) fr = (T)1 - (T)1 / (T)16777216;
        if (fz >= (T)1) fz = (T)1 - (T)1 / (T)16777216;
        if (fr < (T)0) fr = (T)0;
        if (fz < (T)0) fz = (T)0;
        const int64_t d = off + k;
        store_pos(S, d, true, i, j, fr, fz);
        S.vr[d] = (T)vr[k];
        S.vt[d] = (T)vt[k];
        S.vz[d] = (T)vz[k];
        S.id[d] = id[k];
    }
}

template <typename T>
void launch_load(SpeciesDev<T> sp, int64_t offset, const double *r, const double *z,
                 const double *vr, const double *vt, const double *vz, const uint32_t *id,
                 int64_t n, int32_t nr, int32_t nz, double dr, double dz, hipStream_t s)
{
    int blocks = (int)((n + 255) / 256);
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL((k_load<T>), dim3(blocks), dim3(256), 0, s, sp, offset, r, z, vr, vt, vz,
                       id, n, nr, nz, dr, dz);
}

template void launch_push<float>(const PushParams<float> &, int, int, hipStream_t);
template void launch_push<double>(const PushParams<double> &, int, int, hipStream_t);
template void launch_push_b<float>(const PartBatch<float> &, int, hipStream_t);
template void launch_push_b<double>(const PartBatch<double> &, int, hipStream_t);
template void launch_begin_b<float>(const PartBatch<float> &, hipStream_t);
template void launch_begin_b<double>(const PartBatch<double> &, hipStream_t);
template void launch_events_b<float>(const PartBatch<float> &, hipStream_t);
template void launch_events_b<double>(const PartBatch<double> &, hipStream_t);
template void launch_children_b<float>(const PartBatch<float> &, hipStream_t);
template void launch_children_b<double>(const PartBatch<double> &, hipStream_t);
template void launch_finalize_b<float>(const PartBatch<float> &, hipStream_t);
template void launch_finalize_b<double>(const PartBatch<double> &, hipStream_t);
template void launch_events<float>(const EventParams<float> &, hipStream_t);
template void launch_events<double>(const EventParams<double> &, hipStream_t);
template void launch_children<float>(const ChildParams<float> &, hipStream_t);
template void launch_children<double>(const ChildParams<double> &, hipStream_t);
template void launch_load<float>(SpeciesDev<float>, int64_t, const double *, const double *,
                                 const double *, const double *, const double *,
                                 const uint32_t *, int64_t, int32_t, int32_t, double, double,
                                 hipStream_t);
template void launch_load<double>(SpeciesDev<double>, int64_t, const double *, const double *,
                                  const double *, const double *, const double *,
                                  const uint32_t *, int64_t, int32_t, int32_t, double, double,
                                  hipStream_t);

}  // namespace pic
