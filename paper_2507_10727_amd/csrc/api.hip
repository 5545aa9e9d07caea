// Host side of the libpic.so C ABI (include/pic.h): configuration checks,
// workspace layout, set-up tables, and the per-step launch sequence.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "cnn.h"
#include "common.h"

using namespace pic;

namespace {

std::string g_init_error;

struct Buf {
    int32_t *key;
    void *fr, *fz, *vr, *vt, *vz;
    uint32_t *id;
};

struct LevelShape {
    int nr, nz;
    double lr, lz;
};

}  // namespace

struct pic_handle {
    pic_config cfg;
    std::string err;
    hipStream_t stream = nullptr;
    int device = 0;                 // the GPU current at pic_init
    char *ws = nullptr;
    int64_t ws_bytes = 0;
    int prec = PIC_F32;
    size_t ts = 4;
    Buf buf[2][2];
    int cur[2] = {0, 0};
    int64_t cap[2] = {0, 0};
    void *node = nullptr;
    void *q[2] = {nullptr, nullptr};
    DevScalars *sc = nullptr;
    void *child = nullptr;
    int32_t child_cap = 0;
    void *nu = nullptr;
    void *cold = nullptr;
    int2 *mcc_q = nullptr, *see_q = nullptr;
    int32_t ev_cap = 0;
    FieldDev f;
    int32_t *hist = nullptr, *block_sums = nullptr;
    double *diag_partials = nullptr;
    int diag_blocks = 0;
    unsigned long long *live = nullptr;
    std::vector<LevelShape> levels;
    double numax = 0.0;
    unsigned long long t_null = 0, t_see[2] = {0, 0};
    int64_t host_count[2] = {0, 0};
    int steps_since_sort = 0;
    int ion_sort_phase = 0;         // electron sorts since the last ion sort
    pic_poisson_stats last = {};
    double rho = 0.15, rel0_est = 1e-2;
    struct PassGraph {
        const void *phi, *q0, *q1;
        int n_iter, mode;
        hipGraphExec_t exec;
    };
    std::vector<PassGraph> graphs;
    bool use_graphs = false;        // replay each solve pass from a captured graph
    // learned preconditioner
    PcNet net;
    bool pc_on = false;
    int pmode = PIC_MGCG;
    int64_t n_unknown = 0;
    double rho_pc = 0.5, rho_cg = 0.9;
    FastSolve fs = {};              // direct sine-transform solve (PIC_DIRECT)
    bool fs_on = false;
    RunSolve *rsolve = nullptr;     // descriptor of the batched field update
    char *part_desc = nullptr;      // RunParticles for each pair of current particle
                                    // buffers (an ensemble's one-launch particle kernels)
    // launch shape of the particle kernel (autotuned): total blocks and the
    // weight of an electron against an ion when splitting them
    int push_blocks = 1024;
    double push_e_weight = 1.0;
    // plasma diagnostics buffers and the cathode ion-energy record
    // (ied_nbins = 0: not recorded)
    PlasmaDev pd = {};
    int32_t ied_nbins = 0;
    double ied_emax = 0.0, ied_r0 = 0.0, ied_r1 = 0.0;
    bool mg_one_level = false;      // V-cycle with one kernel per grid level
    // pinned host block the field solve reads its status and inner residuals
    // back into (a copy to pageable memory is staged and synchronous)
    double *pinned = nullptr;
    hipEvent_t rb_done = nullptr;   // recorded after the copies; the host spins on it
    int32_t host_flags = 0;
    double check_rtol2 = 0.0;       // a step's direct solve left its check to the circuit kernel
    bool timers_on = false;
    bool timers_push_only = false;  // time the particle kernel alone
    std::vector<std::tuple<int, hipEvent_t, hipEvent_t>> pending;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> free_events;
    pic_timers timers = {};
};

namespace {

pic_status fail(pic_handle *h, pic_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    if (h) h->err = buf;
    else g_init_error = buf;
    return st;
}

#define HIPCHECK(h, call)                                                                   \
    do {                                                                                    \
        hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail((h), PIC_EHIP, "%s failed: %s", #call, hipGetErrorString(e_));      \
    } while (0)

// Multigrid level shapes: halve while both cell counts are even and the
// smaller one exceeds 4.
int coarse_unknowns(const pic_config &c, const LevelShape &s)
{
    int n = 0;
    for (int j = 0; j <= s.nz; ++j)
        for (int i = 0; i <= s.nr; ++i)
            if (host_node_kind(s.nr, s.nz, c.lr, c.cathode_rmax, i, j) == 0) ++n;
    return n;
}

// Multigrid levels: halve while both cell counts are even and the level
// still has more than MG_DENSE_MAX unknowns; the coarsest level is solved
// exactly with its dense inverse, one parallel matrix-vector product in
// place of the barrier-separated sweeps of the levels below it.  The bound
// keeps the inverse small: the coarse-level kernel runs on one CU, which
// reads it from L2 at a few hundred GB/s.
constexpr int MG_DENSE_MAX = 200;

std::vector<LevelShape> mg_shapes(const pic_config &c)
{
    std::vector<LevelShape> v;
    LevelShape s{c.nr, c.nz, c.lr, c.lz};
    v.push_back(s);
    while ((int)v.size() < MAX_LEVELS && (s.nr % 2 == 0) && (s.nz % 2 == 0) &&
           std::min(s.nr, s.nz) > 4 && coarse_unknowns(c, s) > MG_DENSE_MAX) {
        s.nr /= 2;
        s.nz /= 2;
        v.push_back(s);
    }
    return v;
}

// The coarse levels small enough for one workgroup (<= 2600 nodes on the
// first of them) run in the tail kernel, all in LDS; the coarsest level
// always does.
int tail_first(const std::vector<LevelShape> &shapes)
{
    const int nl = (int)shapes.size();
    for (int l = 0; l < nl; ++l) {
        int64_t words = (int64_t)(shapes[l].nr + 1) * (shapes[l].nz + 1);
        const int64_t top = words;
        for (int m = l; m < nl; ++m)
            words += 2 * (int64_t)(shapes[m].nr + 1) * (shapes[m].nz + 1);
        if (top <= 2600 && words * 4 <= MG_TAIL_LDS_MAX) return l;
    }
    return nl - 1;
}

pic_status validate(const pic_config *c, pic_handle *h)
{
    if (!c) return fail(h, PIC_EINVAL, "config is NULL");
    if (c->nr < 2 || c->nz < 2 || c->nr > 65535 || c->nz > 32767)
        return fail(h, PIC_EINVAL, "grid %d x %d outside [2, 65535] x [2, 32767]", c->nr, c->nz);
    if (c->precision == PIC_F32 && (c->nr > POS_MAX_CELLS || c->nz > POS_MAX_CELLS))
        return fail(h, PIC_EINVAL, "FP32 state packs the cell into %d bits: at most %d cells per axis",
                    31 - POS_BITS, POS_MAX_CELLS);
    if (!(c->lr > 0) || !(c->lz > 0) || !(c->dt > 0))
        return fail(h, PIC_EINVAL, "lr, lz and dt must be positive");
    if (c->scheme != PIC_MC && c->scheme != PIC_EC) return fail(h, PIC_EINVAL, "bad scheme");
    if (c->precision != PIC_F32 && c->precision != PIC_F64)
        return fail(h, PIC_EINVAL, "bad precision");
    if (c->circuit != PIC_FIXED_V && c->circuit != PIC_RESISTOR)
        return fail(h, PIC_EINVAL, "bad circuit");
    if (c->circuit == PIC_RESISTOR && !(c->r_ext > 0))
        return fail(h, PIC_EINVAL, "r_ext must be positive");
    if (!(c->cathode_rmax >= 0) || c->cathode_rmax > c->lr)
        return fail(h, PIC_EINVAL, "cathode_rmax outside [0, lr]");
    if (!c->sigma || c->n_table < 2 || !(c->de_table > 0))
        return fail(h, PIC_EINVAL, "cross-section table missing or too short");
    if (!c->b_r || !c->b_z) return fail(h, PIC_EINVAL, "magnetic field arrays missing");
    for (int s = 0; s < 2; ++s) {
        if (!(c->m[s] > 0) || !(c->w[s] > 0))
            return fail(h, PIC_EINVAL, "species %d: mass and weight must be positive", s);
        if (c->capacity[s] < 0 || c->capacity[s] > (int64_t)2000000000)
            return fail(h, PIC_EINVAL, "species %d: capacity out of range", s);
    }
    if (c->sort_every < 1) return fail(h, PIC_EINVAL, "sort_every must be >= 1");
    if (!(c->poisson_rtol > 0) || c->poisson_maxit < 1 || c->poisson_maxit > MAX_PCG)
        return fail(h, PIC_EINVAL, "poisson_rtol > 0 and 1 <= poisson_maxit <= %d required", MAX_PCG);
    if (c->poisson_mode != PIC_MGCG && c->poisson_mode != PIC_LEARNED &&
        c->poisson_mode != PIC_CG && c->poisson_mode != PIC_DIRECT)
        return fail(h, PIC_EINVAL, "poisson_mode must be PIC_MGCG, PIC_LEARNED, PIC_CG or PIC_DIRECT");
    if (c->poisson_mode == PIC_DIRECT) {
        if (host_node_kind(c->nr, c->nz, c->lr, c->cathode_rmax, c->nr - 1, 0) != 1)
            return fail(h, PIC_EINVAL,
                        "PIC_DIRECT needs the cathode to cover the z = 0 row (cathode_rmax > "
                        "(nr - 1) dr): with a Neumann block the field equation does not separate");
        if (c->nr > 1024 || c->nz > 2048)
            return fail(h, PIC_EINVAL, "PIC_DIRECT supports at most 1024 x 2048 cells");
    }
    if (c->pc_batch < 0 || c->pc_batch > 64)
        return fail(h, PIC_EINVAL, "pc_batch outside [0, 64]");
    if (c->pc_batch > 0 || c->poisson_mode == PIC_LEARNED) {
        PcNet t;
        pc_describe(t, c->nr, c->nz, 1);
        if (!pc_fits(t))
            return fail(h, PIC_EINVAL, "grid too narrow for the learned preconditioner's "
                                       "convolution blocks (their input patch exceeds LDS)");
    }
    if (c->pc_maxit < 0 || c->pc_maxit > MAX_PCG)
        return fail(h, PIC_EINVAL, "pc_maxit outside [0, %d]", MAX_PCG);
    if (c->gamma_i < 0 || c->p_gas < 0 || !(c->t_gas > 0))
        return fail(h, PIC_EINVAL, "gamma_i, p_gas >= 0 and t_gas > 0 required");
    if (!(c->gamma_e >= 0) || !(c->n_meta >= 0) || !(c->e_iz_meta > 0))
        return fail(h, PIC_EINVAL, "gamma_e, n_meta >= 0 and e_iz_meta > 0 required");
    if (c->deposit_fixed != 0 && c->deposit_fixed != 1)
        return fail(h, PIC_EINVAL, "deposit_fixed must be 0 or 1");
    if (c->deposit_fixed && c->precision != PIC_F64)
        return fail(h, PIC_EINVAL, "the fixed-point deposit needs FP64 state");
    if (c->pc_pre != 0 && c->pc_pre != 1)
        return fail(h, PIC_EINVAL, "pc_pre must be 0 or 1");
    for (int k = 0; k < 3; ++k)
        if (c->wall_bc[k] != PIC_ABSORB && c->wall_bc[k] != PIC_REFLECT)
            return fail(h, PIC_EINVAL, "bad wall_bc[%d]", k);
    auto lv = mg_shapes(*c);
    const int cu = coarse_unknowns(*c, lv.back());
    if (cu > 2048)
        return fail(h, PIC_EINVAL,
                    "grid %d x %d does not coarsen below 2048 unknowns (coarsest %d x %d)", c->nr,
                    c->nz, lv.back().nr, lv.back().nz);
    const LevelShape &top = lv[tail_first(lv)];
    if ((int64_t)(top.nr + 1) * (top.nz + 1) > MG_TAIL_NODES_MAX)
        return fail(h, PIC_EINVAL,
                    "grid %d x %d: its coarse levels start at %d x %d cells, above the %d nodes "
                    "one workgroup solves",
                    c->nr, c->nz, top.nr, top.nz, MG_TAIL_NODES_MAX);
    return PIC_OK;
}

constexpr int64_t PART_DESC_BYTES =
    ((int64_t)std::max(sizeof(RunParticles<float>), sizeof(RunParticles<double>)) + 255) & ~255;

// Workspace layout.  With base == nullptr only the size is computed.
struct Carver {
    char *base;
    int64_t off = 0;
    template <typename P>
    P *take(int64_t bytes)
    {
        off = (off + 255) & ~(int64_t)255;
        P *p = base ? (P *)(base + off) : nullptr;
        off += bytes;
        return p;
    }
};

int64_t layout(const pic_config &c, char *base, pic_handle *h)
{
    Carver cv{base};
    const size_t ts = (c.precision == PIC_F64) ? 8 : 4;
    const int64_t nodes = (int64_t)(c.nr + 1) * (c.nz + 1);
    const int64_t cap0 = c.capacity[0], cap1 = c.capacity[1];
    const int32_t child_cap = (int32_t)std::max<int64_t>(1 << 16, (cap0 + cap1) / 64);
    DevScalars *sc = cv.take<DevScalars>(sizeof(DevScalars));
    Buf bufs[2][2];
    for (int s = 0; s < 2; ++s) {
        // slots rounded up to 4: the particle kernel moves 4 consecutive slots
        const int64_t cap = ((s ? cap1 : cap0) + 3) & ~(int64_t)3;
        for (int b = 0; b < 2; ++b) {
            Buf &B = bufs[s][b];
            B.key = cv.take<int32_t>(cap * 4);
            B.fr = cv.take<char>(cap * ts);
            B.fz = cv.take<char>(cap * ts);
            B.vr = cv.take<char>(cap * ts);
            B.vt = cv.take<char>(cap * ts);
            B.vz = cv.take<char>(cap * ts);
            B.id = cv.take<uint32_t>(cap * 4);
        }
    }
    void *node = cv.take<char>(nodes * 4 * ts);
    void *q0 = cv.take<char>(nodes * ts);
    void *q1 = cv.take<char>(nodes * ts);
    const size_t child_bytes = (ts == 8) ? sizeof(Child<double>) : sizeof(Child<float>);
    void *child = cv.take<char>((int64_t)child_cap * child_bytes);
    void *nu = cv.take<char>((int64_t)4 * c.n_table * ts);
    void *cold = cv.take<char>(sizeof(PushCold<double>));
    const int64_t ev_cap = std::max<int64_t>(1024, std::max(cap0, cap1));
    int2 *mcc_q = cv.take<int2>(ev_cap * 8);
    int2 *see_q = cv.take<int2>(ev_cap * 8);
    FieldDev f;
    memset(&f, 0, sizeof(f));
    f.nr = c.nr;
    f.nz = c.nz;
    f.dr = c.lr / c.nr;
    f.dz = c.lz / c.nz;
    f.ce64 = cv.take<double>(nodes * 8);
    f.cn64 = cv.take<double>(nodes * 8);
    f.kind = cv.take<uint8_t>(nodes);
    f.phi = cv.take<double>(nodes * 8);
    f.phi0 = cv.take<double>(nodes * 8);
    f.phi_l = cv.take<double>(nodes * 8);
    f.phi0_prev = cv.take<double>(nodes * 8);
    f.r64 = cv.take<double>(nodes * 8);
    f.b_r = cv.take<double>(nodes * 8);
    f.b_z = cv.take<double>(nodes * 8);
    f.vdep = cv.take<double>(nodes * 8);
    f.e32 = cv.take<float>(nodes * 4);
    f.q32 = cv.take<float>(nodes * 4);
    f.p32[0] = cv.take<float>(nodes * 4);
    f.p32[1] = cv.take<float>(nodes * 4);
    f.q32b = cv.take<float>(nodes * 4);
    f.r32b = cv.take<float>(nodes * 4);
    f.w32 = cv.take<float>(nodes * 4);
    f.cg_acc = cv.take<double>((int64_t)MAX_PCG * CG_ACC_PER_ITER * 8);
    auto shapes = mg_shapes(c);
    MGHier &H = f.mg;
    H.nlevels = (int)shapes.size();
    for (int l = 0; l < H.nlevels; ++l) {
        const int64_t nl = (int64_t)(shapes[l].nr + 1) * (shapes[l].nz + 1);
        MGLevel &L = H.lv[l];
        L.nr = shapes[l].nr;
        L.nz = shapes[l].nz;
        L.cath = 0;
        for (int i = 0; i < L.nr; ++i)
            if (host_node_kind(L.nr, L.nz, c.lr, c.cathode_rmax, i, 0) == 1) L.cath = i + 1;
        const double dr = c.lr / L.nr, dz = c.lz / L.nz;
        L.dz = (float)dz;
        L.dr2dz = (float)(dr * dr / dz);
        L.b = cv.take<float>(nl * 4);
        L.xd = cv.take<float>(nl * 4);
        L.xu = cv.take<float>(nl * 4);
    }
    const int first = tail_first(shapes);
    H.tail.first = first;
    H.tail.last = H.nlevels - 1;
    H.tail.tmp_size = (shapes[first].nr + 1) * (shapes[first].nz + 1);
    int64_t words = H.tail.tmp_size;
    for (int m = 0; m < MAX_LEVELS; ++m) H.tail.offx[m] = H.tail.offb[m] = 0;
    for (int m = first; m < H.nlevels; ++m) {
        const int64_t nm = (int64_t)(shapes[m].nr + 1) * (shapes[m].nz + 1);
        H.tail.offx[m] = (int32_t)words;
        H.tail.offb[m] = (int32_t)(words + nm);
        words += 2 * nm;
    }
    H.tail_lds_bytes = (int32_t)(words * 4);
    for (int l = 0; l < H.nlevels; ++l) H.tail.L[l] = H.lv[l];
    const int cu = coarse_unknowns(c, shapes.back());
    H.tail.ninv = cu;
    H.tail.inv = cv.take<float>((int64_t)cu * cu * 4);
    H.tail.map = cv.take<int32_t>((int64_t)cu * 4);
    const int32_t nbins = c.nr * c.nz;
    int32_t *hist = cv.take<int32_t>((int64_t)nbins * 4);
    int32_t *bsums = cv.take<int32_t>((int64_t)((nbins + 1023) / 1024) * 4);
    const int dblocks = 256;
    double *dpart = cv.take<double>((int64_t)dblocks * 6 * 8);
    unsigned long long *live = cv.take<unsigned long long>(2 * 8);
    RunSolve *rsolve = cv.take<RunSolve>(sizeof(RunSolve));
    char *part_desc = cv.take<char>(4 * PART_DESC_BYTES);
    // plasma diagnostics: moments of both species, cell maps, band profiles
    PlasmaDev pd;
    {
        const int64_t ncell = (int64_t)c.nr * c.nz;
        pd.mom[0] = cv.take<double>(5 * ncell * 8);
        pd.mom[1] = cv.take<double>(5 * ncell * 8);
        pd.maps = cv.take<double>(4 * ncell * 8);
        pd.prof = cv.take<double>(3 * (int64_t)(c.nz + 1) * 8);
        pd.out = cv.take<char>(sizeof(PlasmaOut));
        pd.ied = cv.take<unsigned long long>((IED_MAX_BINS + 1) * 8);
    }
    // direct solve: sine transform, right-hand side and its transform, tables
    FastSolve fs = {};
    const bool fs_on = c.poisson_mode == PIC_DIRECT;
    if (fs_on) {
        const int64_t Mp = fs_pad(c.nz - 1), Np = fs_pad(c.nr);
        fs.S = cv.take<double>(Mp * Mp * 8);
        fs.b = cv.take<double>(Mp * Np * 8);
        fs.bh = cv.take<double>(Mp * Np * 8);
        fs.ce1 = cv.take<double>(Np * 8);
        fs.cn1 = cv.take<double>(Np * 8);
        fs.lam = cv.take<double>(Mp * 8);
    }
    // learned preconditioner: network, Adam state and activations
    const bool pc_on = c.pc_batch > 0 || c.poisson_mode == PIC_LEARNED;
    PcNet net;
    char *pc_base = nullptr;
    if (pc_on) {
        pc_describe(net, c.nr, c.nz, std::max(1, c.pc_batch));
        pc_base = cv.take<char>(pc_bytes(net));
    }
    if (h) {
        h->fs = fs;
        h->fs_on = fs_on;
        h->rsolve = rsolve;
        h->part_desc = part_desc;
        h->pd = pd;
        h->pc_on = pc_on;
        if (pc_on) {
            h->net = net;
            pc_bind(h->net, pc_base);
        }
        h->sc = sc;
        for (int s = 0; s < 2; ++s)
            for (int b = 0; b < 2; ++b) h->buf[s][b] = bufs[s][b];
        h->node = node;
        h->q[0] = q0;
        h->q[1] = q1;
        h->child = child;
        h->child_cap = child_cap;
        h->nu = nu;
        h->cold = cold;
        h->mcc_q = mcc_q;
        h->see_q = see_q;
        h->ev_cap = (int32_t)ev_cap;
        h->f = f;
        h->hist = hist;
        h->block_sums = bsums;
        h->diag_partials = dpart;
        h->diag_blocks = dblocks;
        h->live = live;
        h->levels = shapes;
    }
    return cv.off + 256;
}

template <typename T>
SpeciesDev<T> species_dev(const Buf &b)
{
    return SpeciesDev<T>{b.key, (T *)b.fr, (T *)b.fz, (T *)b.vr, (T *)b.vt, (T *)b.vz, b.id};
}

// Words of the current buffer that are negative exactly for absorbed slots:
// the key (FP64 state) or the packed z word (FP32 state).
const int32_t *live_key_words(const pic_handle *h, int s)
{
    const Buf &b = h->buf[s][h->cur[s]];
    return h->prec == PIC_F64 ? b.key : (const int32_t *)b.fz;
}

// ---- timers
void timer_begin(pic_handle *h, hipEvent_t *a, int phase)
{
    a[0] = a[1] = nullptr;
    if (!h->timers_on || (h->timers_push_only && phase != 0)) return;
    hipEvent_t e0, e1;
    if (!h->free_events.empty()) {
        e0 = h->free_events.back().first;
        e1 = h->free_events.back().second;
        h->free_events.pop_back();
    } else {
        (void)hipEventCreate(&e0);
        (void)hipEventCreate(&e1);
    }
    (void)hipEventRecord(e0, h->stream);
    a[0] = e0;
    a[1] = e1;
}

void timer_end(pic_handle *h, int phase, hipEvent_t *a)
{
    if (!a[0]) return;
    (void)hipEventRecord(a[1], h->stream);
    h->pending.emplace_back(phase, a[0], a[1]);
}

void timers_collect(pic_handle *h)
{
    for (auto &t : h->pending) {
        hipEvent_t a = std::get<1>(t), b = std::get<2>(t);
        (void)hipEventSynchronize(b);
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, a, b);
        switch (std::get<0>(t)) {
            case 0: h->timers.push_ms += ms; h->timers.push_launches++; break;
            case 1: h->timers.children_ms += ms; break;
            case 2: h->timers.sort_ms += ms; h->timers.sort_launches++; break;
            case 3: h->timers.poisson_ms += ms; h->timers.poisson_solves++; break;
            case 4: h->timers.circuit_ms += ms; break;
            case 5: h->timers.field_ms += ms; break;
        }
        h->free_events.emplace_back(a, b);
    }
    h->pending.clear();
}

// ---- set-up of the multigrid hierarchy and the FP64 operator
pic_status setup_field(pic_handle *h)
{
    const pic_config &c = h->cfg;
    const int64_t nodes = (int64_t)(c.nr + 1) * (c.nz + 1);
    std::vector<double> ce(nodes), cn(nodes), tmp(nodes);
    std::vector<uint8_t> kind(nodes);
    host_couplings(c.nr, c.nz, c.lr, c.lz, eps0(), ce.data(), cn.data());
    for (int j = 0; j <= c.nz; ++j)
        for (int i = 0; i <= c.nr; ++i)
            kind[(int64_t)j * (c.nr + 1) + i] =
                (uint8_t)host_node_kind(c.nr, c.nz, c.lr, c.cathode_rmax, i, j);
    HIPCHECK(h, hipMemcpy((void *)h->f.ce64, ce.data(), nodes * 8, hipMemcpyHostToDevice));
    HIPCHECK(h, hipMemcpy((void *)h->f.cn64, cn.data(), nodes * 8, hipMemcpyHostToDevice));
    HIPCHECK(h, hipMemcpy((void *)h->f.kind, kind.data(), nodes, hipMemcpyHostToDevice));
    h->n_unknown = std::count(kind.begin(), kind.end(), (uint8_t)0);
    if (h->pc_on && pc_kernel_setup() != 0)
        return fail(h, PIC_EHIP, "cannot raise the LDS limit of the convolution kernels");
    host_node_volumes(c.nr, c.nz, c.lr, c.lz, tmp.data());
    HIPCHECK(h, hipMemcpy((void *)h->f.vdep, tmp.data(), nodes * 8, hipMemcpyHostToDevice));
    HIPCHECK(h, hipMemcpy((void *)h->f.b_r, c.b_r, nodes * 8, hipMemcpyHostToDevice));
    HIPCHECK(h, hipMemcpy((void *)h->f.b_z, c.b_z, nodes * 8, hipMemcpyHostToDevice));

    // dense inverse of the coarsest level's operator (couplings / (2 pi eps0))
    {
        MGHier &H = h->f.mg;
        const LevelShape &s = h->levels[H.nlevels - 1];
        const int64_t nl = (int64_t)(s.nr + 1) * (s.nz + 1);
        std::vector<double> a(nl), b(nl);
        const double scale = 2.0 * 3.14159265358979323846;
        host_couplings(s.nr, s.nz, s.lr, s.lz, 1.0 / scale, a.data(), b.data());
        std::vector<int32_t> map;
        std::vector<int> idx(nl, -1);
        const int ld = s.nr + 1;
        for (int64_t n = 0; n < nl; ++n) {
            const int j = (int)(n / ld), i = (int)(n % ld);
            if (host_node_kind(s.nr, s.nz, c.lr, c.cathode_rmax, i, j) == 0) {
                idx[n] = (int)map.size();
                map.push_back((int32_t)n);
            }
        }
        const int m = (int)map.size();
        std::vector<double> A((size_t)m * m, 0.0);
        for (int u = 0; u < m; ++u) {
            const int64_t n = map[u];
            const int j = (int)(n / ld), i = (int)(n % ld);
            double d = 0.0;
            auto add = [&](int64_t nb, double cpl) {
                d += cpl;
                if (idx[nb] >= 0) A[(size_t)u * m + idx[nb]] -= cpl;
            };
            if (i < s.nr) add(n + 1, a[n]);
            if (i > 0) add(n - 1, a[n - 1]);
            if (j < s.nz) add(n + ld, b[n]);
            if (j > 0) add(n - ld, b[n - ld]);
            A[(size_t)u * m + u] += d;
        }
        if (m > 0 && host_dense_inverse(m, A.data()) != 0)
            return fail(h, PIC_EINVAL, "coarsest operator is singular");
        std::vector<float> Af(A.begin(), A.end());
        if (m > 0) {
            HIPCHECK(h, hipMemcpy((void *)H.tail.inv, Af.data(), (size_t)m * m * 4,
                                  hipMemcpyHostToDevice));
            HIPCHECK(h, hipMemcpy((void *)H.tail.map, map.data(), (size_t)m * 4,
                                  hipMemcpyHostToDevice));
        }
        H.tail.ninv = m;
        for (int l = 0; l < H.nlevels; ++l) {
            const int64_t n = (int64_t)(H.lv[l].nr + 1) * (H.lv[l].nz + 1);
            launch_zero(H.lv[l].b, n * 4, h->stream);
            launch_zero(H.lv[l].xd, n * 4, h->stream);
            launch_zero(H.lv[l].xu, n * 4, h->stream);
        }
        if (mg_tail_setup(H) != 0)
            return fail(h, PIC_EHIP, "cannot reserve %d bytes of LDS for the coarse levels",
                        H.tail_lds_bytes);
    }
    if (h->fs_on) {
        if (!fs_separable(c.nr, c.nz, ce.data(), cn.data(), kind.data()))
            return fail(h, PIC_EINVAL, "the field equation of this grid does not separate");
        const int Mp = fs_pad(c.nz - 1), Np = fs_pad(c.nr);
        std::vector<double> S((size_t)Mp * Mp), ce1(Np, 0.0), cn1(Np, 0.0), lam(Mp);
        fs_tables(c.nr, c.nz, ce.data(), cn.data(), S.data(), ce1.data(), cn1.data(), lam.data());
        HIPCHECK(h, hipMemcpy((void *)h->fs.S, S.data(), S.size() * 8, hipMemcpyHostToDevice));
        HIPCHECK(h, hipMemcpy((void *)h->fs.ce1, ce1.data(), Np * 8, hipMemcpyHostToDevice));
        HIPCHECK(h, hipMemcpy((void *)h->fs.cn1, cn1.data(), Np * 8, hipMemcpyHostToDevice));
        HIPCHECK(h, hipMemcpy((void *)h->fs.lam, lam.data(), Mp * 8, hipMemcpyHostToDevice));
        launch_zero(h->fs.b, (int64_t)Mp * Np * 8, h->stream);
        launch_zero(h->fs.bh, (int64_t)Mp * Np * 8, h->stream);
    }
    launch_zero(h->f.e32, nodes * 4, h->stream);
    launch_zero(h->f.q32b, nodes * 4, h->stream);
    launch_zero(h->f.r32b, nodes * 4, h->stream);
    launch_zero(h->f.w32, nodes * 4, h->stream);
    launch_zero(h->f.p32[0], nodes * 4, h->stream);
    launch_zero(h->f.p32[1], nodes * 4, h->stream);
    launch_zero(h->f.q32, nodes * 4, h->stream);
    return PIC_OK;
}

// ---- field solve: FP64 iterative refinement around an FP32 MG-PCG
//
// A pass: FP64 residual r = q - K phi (norm kept on the device), r / ||r||
// to FP32, a fixed number of conjugate-gradient iterations on the FP32
// operator K / (2 pi eps0) preconditioned by one multigrid V-cycle each,
// phi += e ||r|| / (2 pi eps0) in FP64, and the FP64 residual of the result,
// read back with the step's flags and counts in one copy (the pass's only
// synchronization).  The iteration count is predicted from earlier solves
// and, for a further pass, from the convergence rate the last pass reached.
struct SolveReadback {
    double rr, bb, rr0;
    int32_t flags, pad;
    int64_t count[2];
};

// With hist, also the inner iterations' squared residuals of the pass (the
// FP32 residual starts at unit norm), in the same synchronization.
constexpr size_t PINNED_BYTES =
    sizeof(SolveReadback) + (RES_SLOT_WORDS + MAX_PCG) * sizeof(double);

pic_status readback(pic_handle *h, SolveReadback *rb, double *hist = nullptr, int n_hist = 0)
{
    static_assert(sizeof(SolveReadback) == 48, "readback layout");
    char *pin = (char *)h->pinned;
    double *slots = (double *)(pin + sizeof(SolveReadback));
    char *hist_pin = pin + sizeof(SolveReadback) + RES_SLOT_WORDS * sizeof(double);
    HIPCHECK(h, hipMemcpyAsync(pin, &h->sc->res_rr, sizeof(SolveReadback), hipMemcpyDeviceToHost,
                               h->stream));
    HIPCHECK(h, hipMemcpyAsync(slots, h->sc->res_slots, RES_SLOT_WORDS * sizeof(double),
                               hipMemcpyDeviceToHost, h->stream));
    if (hist && n_hist > 0)
        HIPCHECK(h, hipMemcpyAsync(hist_pin, h->sc->pcg_rr, (size_t)n_hist * 8,
                                   hipMemcpyDeviceToHost, h->stream));
    // the solve's only synchronization sits on the step's critical path:
    // poll for it rather than let the runtime block and be woken
    HIPCHECK(h, hipEventRecord(h->rb_done, h->stream));
    hipError_t q;
    while ((q = hipEventQuery(h->rb_done)) == hipErrorNotReady) {
    }
    HIPCHECK(h, q);
    memcpy(rb, pin, sizeof(SolveReadback));
    // the residual norms are kept in slots (summed in slot order)
    rb->rr = rb->bb = 0.0;
    for (int k = 0; k < ACC_SLOTS; ++k) {
        rb->rr += slots[k * ACC_STRIDE];
        rb->bb += slots[(ACC_SLOTS + k) * ACC_STRIDE];
    }
    if (hist && n_hist > 0) memcpy(hist, hist_pin, (size_t)n_hist * 8);
    h->host_count[0] = rb->count[0];
    h->host_count[1] = rb->count[1];
    h->host_flags = rb->flags;
    return PIC_OK;
}

// Preconditioner of CG iteration k: z = M r on the finest level, r.z into
// pcg_rz[k] (and z_k.q_{k-1} into pcg_zq[k] for the learned one).
// The learned preconditioner's first approximation: a multigrid V-cycle
// (pc_pre = 1) or a red-black Gauss-Seidel pair.
PcPre pc_pre_of(const pic_handle *h)
{
    PcPre p;
    p.H = h->cfg.pc_pre ? &h->f.mg : nullptr;
    p.two_level = !h->mg_one_level;
    return p;
}

void enqueue_precond(pic_handle *h, int mode, int k)
{
    hipStream_t s = h->stream;
    FieldDev &f = h->f;
    const MGHier &H = f.mg;
    if (mode == PIC_LEARNED)
        pc_apply32(h->net, pc_pre_of(h), H.lv[0], h->n_unknown, H.lv[0].b, H.lv[0].xu,
                   k > 0 ? f.q32 : nullptr, &h->sc->pcg_rz[k], &h->sc->pcg_zq[k],
                   &h->sc->pcg_ss[k], s);
    else if (mode == PIC_CG)
        pc_identity32(H.lv[0], H.lv[0].b, H.lv[0].xu, &h->sc->pcg_rz[k], s);
    else
        launch_mg_vcycle(H, &h->sc->pcg_rz[k], s, !h->mg_one_level);
}

// One refinement pass (after the residual that precedes it): scale, n_iter
// preconditioned CG iterations (flexible CG for the learned preconditioner),
// FP64 update and the new residual.
template <typename Q>
void enqueue_pass(pic_handle *h, double *phi, const Q *q0, const Q *q1, int n_iter, int mode)
{
    hipStream_t s = h->stream;
    FieldDev &f = h->f;
    const MGHier &H = f.mg;
    const double inv_2pi_eps0 = 1.0 / (2.0 * 3.14159265358979323846 * eps0());
    const double *zq = (mode == PIC_LEARNED) ? h->sc->pcg_zq : nullptr;
    if (mode == PIC_MGCG && !h->mg_one_level && H.tail.first >= 1) {
        // CG vector work fused into the finest level's V-cycle kernels; the
        // cast clears the pass's slotted dots, the FP64 update sums each
        // iteration's ||r||^2 into pcg_rr for the readback
        launch_cast_scale(f, h->sc, s, f.cg_acc, (int64_t)n_iter * CG_ACC_PER_ITER);
        CgVecs v;
        v.r[0] = H.lv[0].b;
        v.r[1] = f.r32b;
        v.q[0] = f.q32;
        v.q[1] = f.q32b;
        v.w = f.w32;
        v.p = f.p32[0];
        v.e = f.e32;
        v.acc = f.cg_acc;
        v.pq = h->sc->pcg_pq;
        for (int k = 0; k < n_iter; ++k) launch_mg_vcycle_cg(H, v, k, s, true);
        launch_cg_update_last(H, v, n_iter - 1, s);
        launch_update64(f, phi, h->sc, inv_2pi_eps0, s, true, n_iter);
        launch_residual64<Q>(f, phi, q0, q1, h->sc, s, false);
        return;
    }
    // (the cast also clears the pass's CG accumulators: pcg_rz .. pcg_ss)
    launch_cast_scale(f, h->sc, s, h->sc->pcg_rz, 5 * (MAX_PCG + 2));
    enqueue_precond(h, mode, 0);
    for (int k = 0; k < n_iter; ++k) {
        launch_cg_matvec(H, H.lv[0].xu, f.p32[(k + 1) & 1], f.p32[k & 1], f.q32, h->sc->pcg_rz,
                         k, &h->sc->pcg_pq[k], zq, s);
        launch_cg_update(H, f.p32[k & 1], f.q32, f.e32, H.lv[0].b, &h->sc->pcg_rz[k],
                         &h->sc->pcg_pq[k], &h->sc->pcg_rr[k], s);
        if (k + 1 < n_iter) enqueue_precond(h, mode, k + 1);
    }
    launch_update64(f, phi, h->sc, inv_2pi_eps0, s, true);
    launch_residual64<Q>(f, phi, q0, q1, h->sc, s, false);
}

void drop_graphs(pic_handle *h)
{
    for (auto &g : h->graphs) (void)hipGraphExecDestroy(g.exec);
    h->graphs.clear();
}

// The pass's kernels are launched directly, or (pass_graphs tuning) replayed
// from a cached hipGraph per (buffers, iteration count, preconditioner) when
// the stream allows capture.
template <typename Q>
pic_status run_pass(pic_handle *h, double *phi, const Q *q0, const Q *q1, int n_iter, int mode)
{
    if (!h->use_graphs || h->stream == nullptr) {
        enqueue_pass<Q>(h, phi, q0, q1, n_iter, mode);
        return PIC_OK;
    }
    for (auto &g : h->graphs)
        if (g.phi == phi && g.q0 == q0 && g.q1 == q1 && g.n_iter == n_iter && g.mode == mode) {
            HIPCHECK(h, hipGraphLaunch(g.exec, h->stream));
            return PIC_OK;
        }
    hipGraph_t graph;
    if (hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        (void)hipGetLastError();
        h->use_graphs = false;
        enqueue_pass<Q>(h, phi, q0, q1, n_iter, mode);
        return PIC_OK;
    }
    enqueue_pass<Q>(h, phi, q0, q1, n_iter, mode);
    HIPCHECK(h, hipStreamEndCapture(h->stream, &graph));
    hipGraphExec_t exec;
    HIPCHECK(h, hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
    (void)hipGraphDestroy(graph);
    h->graphs.push_back({phi, q0, q1, n_iter, mode, exec});
    HIPCHECK(h, hipGraphLaunch(exec, h->stream));
    return PIC_OK;
}

// FP64-refined solve (extrapolate: start from phi0 extrapolated from the last
// two steps).  With the learned preconditioner, after pc_maxit of its
// iterations without convergence, or a pass that does not lower the
// residual, the remaining passes use the multigrid preconditioner.
template <typename Q>
pic_status solve(pic_handle *h, double *phi, const Q *q0, const Q *q1, double v_cathode,
                 pic_poisson_stats *st, int mode, bool extrapolate = false, bool sync = true)
{
    hipStream_t s = h->stream;
    FieldDev &f = h->f;
    const double rtol = h->cfg.poisson_rtol;
    const int maxit = h->cfg.poisson_maxit;
    const int pc_cap = h->cfg.pc_maxit > 0 ? h->cfg.pc_maxit : maxit;
    if (mode == PIC_LEARNED && !(h->pc_on && h->net.has_weights))
        return fail(h, PIC_ESTATE, "the learned preconditioner has no weights");
    pic_status pe = PIC_OK;
    pic_poisson_stats S = {};
    launch_solve_prep(f, phi, extrapolate, v_cathode, h->sc, s);
    if (mode == PIC_DIRECT) {
        // residual correction with the direct FP64 solve: r = b - K phi,
        // phi += K^-1 r, and the FP64 residual of the result; a step's solve
        // keeps the norms on the device (checked there by the circuit kernel
        // that follows it), a synchronous one corrects again while short of
        // the tolerance
        launch_residual64<Q>(f, phi, q0, q1, h->sc, s, false);
        launch_fast_solve(h->fs, f, phi, h->sc, s);
        launch_residual64<Q>(f, phi, q0, q1, h->sc, s, false);
        S.outer = 1;
        if (!sync) {
            h->check_rtol2 = rtol * rtol;
            S.converged = -1;           // known at the next synchronization
            h->last = S;
            return PIC_OK;
        }
        for (;;) {
            SolveReadback rb;
            pe = readback(h, &rb);
            if (pe != PIC_OK) return pe;
            S.rel_res = rb.bb > 0.0 ? std::sqrt(rb.rr / rb.bb) : 0.0;
            S.converged = (std::isfinite(S.rel_res) && S.rel_res <= rtol) ? 1 : 0;
            if (S.converged || !std::isfinite(S.rel_res) || S.outer == 3) break;
            launch_fast_solve(h->fs, f, phi, h->sc, s);
            launch_residual64<Q>(f, phi, q0, q1, h->sc, s, false);
            S.outer++;
        }
        h->last = S;
        if (st) *st = S;
        if (!std::isfinite(S.rel_res)) return fail(h, PIC_ENAN, "non-finite residual in the field solve");
        if (!S.converged)
            return fail(h, PIC_ENOCONV, "direct field solve left relative residual %.3e (target %.1e)",
                        S.rel_res, rtol);
        return PIC_OK;
    }
    launch_residual64<Q>(f, phi, q0, q1, h->sc, s, false);
    auto rate = [&]() -> double & {
        return mode == PIC_LEARNED ? h->rho_pc : (mode == PIC_CG ? h->rho_cg : h->rho);
    };
    // iterations for a target reduction at the measured rate; one FP32 pass
    // is asked for at most 1e-6 (about what single precision delivers)
    auto iters_for = [&](double rel_now) {
        const double target = std::max(0.5 * rtol / rel_now, 1e-6);
        if (target >= 1.0) return 1;
        const int n = (int)std::ceil(std::log(target) / std::log(rate()));
        return std::max(1, std::min(n, 64));
    };
    double rel_now = h->rel0_est;
    int n_iter = iters_for(rel_now);
    const int max_pass = 24;
    for (int pass = 0;; ++pass) {
        if (pass == max_pass) break;
        int left;
        if (mode == PIC_LEARNED) {
            left = pc_cap - S.pc_iterations;
            if (left <= 0) {
                mode = PIC_MGCG;
                S.fell_back = 1;
                n_iter = iters_for(rel_now);
                left = maxit;
            }
        } else {
            left = maxit - (S.iterations - S.pc_iterations);
        }
        if (left <= 0) break;
        n_iter = std::max(1, std::min(n_iter, left));
        pe = run_pass<Q>(h, phi, q0, q1, n_iter, mode);
        if (pe != PIC_OK) return pe;
        S.iterations += n_iter;
        if (mode == PIC_LEARNED) S.pc_iterations += n_iter;
        S.outer++;
        SolveReadback rb;
        double hist[MAX_PCG];
        pic_status e = readback(h, &rb, hist, n_iter);
        if (e != PIC_OK) return e;
        if (!std::isfinite(rb.rr) || !std::isfinite(rb.bb)) {
            S.rel_res = NAN;
            h->last = S;
            if (st) *st = S;
            return fail(h, PIC_ENAN, "non-finite residual in the field solve");
        }
        if (rb.bb == 0.0) {
            launch_zero_unknowns(f, phi, s);
            S.rel_res = 0.0;
            S.converged = 1;
            break;
        }
        const double rel0 = std::sqrt(rb.rr0 / rb.bb), rel = std::sqrt(rb.rr / rb.bb);
        S.rel_res = rel;
        rel_now = rel;
        if (pass == 0 && rel0 > 0.0) h->rel0_est = rel0;
        // per-iteration rate from the inner residuals: the iterations the
        // pass needed for its target, else the average over the pass
        {
            const double target = std::max(0.5 * rtol / std::max(rel0, 1e-300), 1e-6);
            int hit = -1;
            for (int k = 0; k < n_iter; ++k)
                if (std::sqrt(std::max(hist[k], 0.0)) <= target) {
                    hit = k;
                    break;
                }
            double est;
            if (hit >= 0) est = std::pow(target, 1.0 / (hit + 1));
            else est = std::pow(std::sqrt(std::max(hist[n_iter - 1], 1e-300)), 1.0 / n_iter);
            if (std::isfinite(est) && est > 0.0) rate() = std::min(std::max(est, 0.01), 0.97);
        }
        if (rel <= rtol) {
            S.converged = 1;
            break;
        }
        if (mode == PIC_LEARNED && !(rel < rel0)) {
            mode = PIC_MGCG;
            S.fell_back = 1;
        }
        n_iter = iters_for(rel);
    }
    h->last = S;
    if (st) *st = S;
    if (!S.converged)
        return fail(h, PIC_ENOCONV, "field solve stopped at relative residual %.3e (target %.1e)",
                    S.rel_res, rtol);
    return PIC_OK;
}

template <typename T>
PushCold<T> push_cold(pic_handle *h)
{
    const pic_config &c = h->cfg;
    PushCold<T> C;
    memset(&C, 0, sizeof(C));
    C.child = (Child<T> *)h->child;
    C.child_cap = h->child_cap;
    C.nu = (const T *)h->nu;
    C.n_table = c.n_table;
    C.inv_de = (T)(1.0 / c.de_table);
    C.numax = (T)h->numax;
    C.t_see[0] = h->t_see[0];
    C.t_see[1] = h->t_see[1];
    const double qe = 1.602176634e-19;
    C.e_of_v2 = (T)(0.5 * c.m[0] / qe);
    C.v2_of_e = (T)(2.0 * qe / c.m[0]);
    C.two_m_over_M = (T)(2.0 * c.m[0] / c.m[1]);
    C.e_exc = (T)c.e_exc;
    C.e_iz = (T)c.e_iz;
    C.e_iz_meta = (T)c.e_iz_meta;
    C.sig_ion = (T)std::sqrt(1.380649e-23 * c.t_gas / c.m[1]);
    for (int s = 0; s < 2; ++s) C.qw64[s] = c.q[s] * c.w[s];
    for (int k = 0; k < 3; ++k) C.wall_bc[k] = c.wall_bc[k];
    C.cathode_rmax = (T)c.cathode_rmax;
    return C;
}

template <typename T>
PushParams<T> push_params(pic_handle *h, int deposit_only)
{
    const pic_config &c = h->cfg;
    PushParams<T> P;
    memset(&P, 0, sizeof(P));
    for (int s = 0; s < 2; ++s) {
        P.sp[s] = species_dev<T>(h->buf[s][h->cur[s]]);
        P.q[s] = (T *)h->q[s];
        P.hqm[s] = (T)(0.5 * c.q[s] / c.m[s] * c.dt);
        P.qw[s] = (T)(c.q[s] * c.w[s]);
        P.mw[s] = c.m[s] * c.w[s];
    }
    P.node = (const typename Vec4<T>::type *)h->node;
    P.sc = h->sc;
    P.cold = (const PushCold<T> *)h->cold;
    P.mcc_q = h->mcc_q;
    P.see_q = h->see_q;
    P.ev_cap = h->ev_cap;
    P.t_null = h->t_null;
    P.nr = c.nr;
    P.nz = c.nz;
    P.dr = (T)(c.lr / c.nr);
    P.inv_dr = (T)(c.nr / c.lr);
    P.inv_dz = (T)(c.nz / c.lz);
    P.dt = (T)c.dt;
    P.frozen_ions = c.frozen_ions;
    P.mcc_on = c.mcc_on;
    for (int s = 0; s < 2; ++s) P.emit[s] = (c.see_on && h->t_see[s] > 0) ? 1 : 0;
    P.any_reflect = (c.wall_bc[0] == PIC_REFLECT || c.wall_bc[1] == PIC_REFLECT ||
                     c.wall_bc[2] == PIC_REFLECT) ? 1 : 0;
    P.deposit_only = deposit_only;
    P.fixed_q = c.deposit_fixed;
    P.ied_on = h->ied_nbins > 0 ? 1 : 0;
    P.key0 = (uint32_t)(c.seed & 0xffffffffu);
    P.key1 = (uint32_t)(c.seed >> 32);
    P.run = c.run;
    return P;
}

// Block split of the fused kernel between the species (electrons weigh a
// little more: they also collide).
void push_grid(pic_handle *h, int *nblk_e, int *nblocks)
{
    const double ne = (double)std::max<int64_t>(h->host_count[0], 1);
    const double ni = (double)std::max<int64_t>(h->host_count[1], 1);
    const int total = h->push_blocks;
    const double w = h->push_e_weight;
    int be = (int)std::lround(total * w * ne / (w * ne + ni));
    be = std::max(1, std::min(total - 1, be));
    int bi = total - be;
    be = std::max(1, (int)std::min<int64_t>(be, (h->host_count[0] + PUSH_CHUNK - 1) / PUSH_CHUNK + 1));
    bi = std::max(1, (int)std::min<int64_t>(bi, (h->host_count[1] + PUSH_CHUNK - 1) / PUSH_CHUNK + 1));
    *nblk_e = be;
    *nblocks = be + bi;
}

template <typename T>
void launch_push_h(pic_handle *h, int deposit_only)
{
    PushParams<T> P = push_params<T>(h, deposit_only);
    int be, nb;
    push_grid(h, &be, &nb);
    P.nblk_e = be;
    launch_push<T>(P, h->cfg.scheme, nb, h->stream);
}

template <typename T>
void sort_species(pic_handle *h, int s)
{
    const int from = h->cur[s], to = 1 - from;
    launch_sort<T>(species_dev<T>(h->buf[s][from]), species_dev<T>(h->buf[s][to]), h->sc, s,
                   h->hist, h->block_sums, h->cfg.nr, h->cfg.nz, h->cap[s], h->stream);
    h->cur[s] = to;
}

// Cell sort (and compaction) of both species; periodic: the step's sort,
// which takes the ions only at every PIC_ION_SORT_EVERY-th call.
template <typename T>
void sort_all(pic_handle *h, bool periodic = false)
{
    hipEvent_t ev[2];
    timer_begin(h, ev, 2);
    sort_species<T>(h, 0);
    if (!periodic || ++h->ion_sort_phase >= PIC_ION_SORT_EVERY) {
        sort_species<T>(h, 1);
        h->ion_sort_phase = 0;
    }
    timer_end(h, 2, ev);
    h->steps_since_sort = 0;
}

pic_status read_scalars(pic_handle *h, DevScalars *out)
{
    HIPCHECK(h, hipMemcpyAsync(out, h->sc, sizeof(DevScalars), hipMemcpyDeviceToHost, h->stream));
    HIPCHECK(h, hipStreamSynchronize(h->stream));
    h->host_count[0] = out->count[0];
    h->host_count[1] = out->count[1];
    return PIC_OK;
}

pic_status check_flags(pic_handle *h)
{
    int32_t flags = 0;
    int64_t counts[2];
    HIPCHECK(h, hipMemcpyAsync(&flags, &h->sc->flags, 4, hipMemcpyDeviceToHost, h->stream));
    HIPCHECK(h, hipMemcpyAsync(counts, h->sc->count, 16, hipMemcpyDeviceToHost, h->stream));
    HIPCHECK(h, hipStreamSynchronize(h->stream));
    h->host_count[0] = counts[0];
    h->host_count[1] = counts[1];
    h->host_flags = flags;
    if (flags & (FLAG_CAPACITY | FLAG_CHILD_OVERFLOW))
        return fail(h, PIC_ECAPACITY, "particle capacity exceeded (flags %d)", flags);
    if (flags & FLAG_NOCONV) {
        // reported once: cleared on the device
        const int32_t keep = flags & ~FLAG_NOCONV;
        HIPCHECK(h, hipMemcpyAsync(&h->sc->flags, &keep, 4, hipMemcpyHostToDevice, h->stream));
        HIPCHECK(h, hipStreamSynchronize(h->stream));
        return fail(h, PIC_ENOCONV, "a direct field solve missed its residual tolerance");
    }
    return PIC_OK;
}

template <typename T>
pic_status field_update(pic_handle *h)
{
    const pic_config &c = h->cfg;
    hipEvent_t ev[2];
    timer_begin(h, ev, 3);
    // the warm start (phi0 extrapolated from the last two steps) is applied
    // by the solve's first kernel
    pic_status st = solve<T>(h, h->f.phi0, (const T *)h->q[0], (const T *)h->q[1], 0.0, nullptr,
                              h->pmode, true, h->pmode != PIC_DIRECT);
    timer_end(h, 3, ev);
    if (st != PIC_OK) return st;
    timer_begin(h, ev, 4);
    launch_circuit<T>(h->f, (const T *)h->q[0], (const T *)h->q[1], h->sc, c.circuit, c.v_fixed,
                      c.v_ext, c.r_ext, c.dt, c.extra_current * c.dt, h->stream, h->check_rtol2);
    h->check_rtol2 = 0.0;
    timer_end(h, 4, ev);
    timer_begin(h, ev, 5);
    launch_field_prep<T>(h->f, (typename Vec4<T>::type *)h->node, h->sc, c.scheme, 0, h->stream);
    timer_end(h, 5, ev);
    return PIC_OK;
}

// Particle phase of a step: begin (clear tallies and node charge), push
// (gather, Boris, walls, candidate queues, deposit), events (collisions,
// emission), children (ids, append, deposit), finalize (counts).
template <typename T>
EventParams<T> event_params(const pic_handle *h)
{
    const pic_config &c = h->cfg;
    EventParams<T> E;
    memset(&E, 0, sizeof(E));
    for (int s = 0; s < 2; ++s) E.sp[s] = species_dev<T>(h->buf[s][h->cur[s]]);
    E.cold = (const PushCold<T> *)h->cold;
    E.sc = h->sc;
    E.mcc_q = h->mcc_q;
    E.see_q = h->see_q;
    E.ev_cap = h->ev_cap;
    E.nr = c.nr;
    E.key0 = (uint32_t)(c.seed & 0xffffffffu);
    E.key1 = (uint32_t)(c.seed >> 32);
    E.run = c.run;
    if (h->ied_nbins > 0) {
        E.ied_hist = h->pd.ied;
        E.ied_emax = h->ied_emax;
        E.ied_r0 = h->ied_r0;
        E.ied_r1 = h->ied_r1;
        E.ied_nbins = h->ied_nbins;
        E.ied_m = c.m[1];
        E.dr = c.lr / c.nr;
    }
    return E;
}

template <typename T>
ChildParams<T> child_params(const pic_handle *h)
{
    const pic_config &c = h->cfg;
    ChildParams<T> C;
    memset(&C, 0, sizeof(C));
    for (int s = 0; s < 2; ++s) {
        C.sp[s] = species_dev<T>(h->buf[s][h->cur[s]]);
        C.cap[s] = h->cap[s];
        C.q[s] = (T *)h->q[s];
        C.qw[s] = (T)(c.q[s] * c.w[s]);
        C.qw64[s] = c.q[s] * c.w[s];
    }
    C.sc = h->sc;
    C.child = (const Child<T> *)h->child;
    C.child_cap = h->child_cap;
    C.nr = c.nr;
    C.fixed_q = c.deposit_fixed;
    return C;
}

template <typename T>
void particle_events(pic_handle *h)
{
    hipEvent_t ev[2];
    timer_begin(h, ev, 1);
    launch_events<T>(event_params<T>(h), h->stream);
    launch_children<T>(child_params<T>(h), h->stream);
    const pic_config &c = h->cfg;
    const double qw64[2] = {c.q[0] * c.w[0], c.q[1] * c.w[1]};
    if (c.deposit_fixed)
        launch_q_from_fixed(h->q[0], h->q[1], (int64_t)(c.nr + 1) * (c.nz + 1), qw64, h->stream);
    launch_finalize_step(h->sc, h->cap, qw64, h->stream);
    timer_end(h, 1, ev);
}

template <typename T>
void particle_phase(pic_handle *h)
{
    const pic_config &c = h->cfg;
    const int64_t nodes = (int64_t)(c.nr + 1) * (c.nz + 1);
    launch_begin_step(h->sc, h->q[0], h->q[1], nodes, (int)sizeof(T), h->stream);
    hipEvent_t ev[2];
    timer_begin(h, ev, 0);
    launch_push_h<T>(h, 0);
    timer_end(h, 0, ev);
    particle_events<T>(h);
}

template <typename T>
pic_status step_one(pic_handle *h)
{
    const pic_config &c = h->cfg;
    if (h->steps_since_sort >= c.sort_every) sort_all<T>(h, true);
    particle_phase<T>(h);
    h->steps_since_sort++;
    if (c.field_solve) {
        pic_status st = field_update<T>(h);
        if (st != PIC_OK) return st;
    } else {
        // keep phi; add the synthetic current to the tally like the circuit does
        if (c.extra_current != 0.0) {
            launch_circuit<T>(h->f, (const T *)h->q[0], (const T *)h->q[1], h->sc, PIC_FIXED_V,
                              0.0, 0.0, 1.0, c.dt, c.extra_current * c.dt, h->stream);
        }
    }
    if (c.field_solve) {
        // (the direct solve does not synchronize: pic_step checks the flags
        // once at the end of the call)
        if (h->pmode != PIC_DIRECT && (h->host_flags & (FLAG_CAPACITY | FLAG_CHILD_OVERFLOW)))
            return fail(h, PIC_ECAPACITY, "particle capacity exceeded (flags %d)", h->host_flags);
        return PIC_OK;
    }
    return check_flags(h);
}

// ---- a step with no host synchronization (for graph capture) ---------------

// The particle part of a step (the ensemble batches the field update).
template <typename T>
pic_status init_typed(pic_handle *h, const pic_species_host *init)
{
    const pic_config &c = h->cfg;
    hipStream_t s = h->stream;
    // collision tables
    std::vector<double> nu((size_t)4 * c.n_table);
    h->numax = host_nu_tables(c, nu.data(), &h->t_null);
    h->t_see[0] = host_see_threshold(c, 0);
    h->t_see[1] = host_see_threshold(c, 1);
    std::vector<T> nut(nu.begin(), nu.end());
    HIPCHECK(h, hipMemcpy(h->nu, nut.data(), nut.size() * sizeof(T), hipMemcpyHostToDevice));
    pic_status st = setup_field(h);
    if (st != PIC_OK) return st;
    {
        PushCold<T> C = push_cold<T>(h);
        HIPCHECK(h, hipMemcpy(h->cold, &C, sizeof(C), hipMemcpyHostToDevice));
    }
    // scalars
    launch_zero(h->sc, sizeof(DevScalars), s);
    HIPCHECK(h, hipStreamSynchronize(s));
    DevScalars sc0;
    memset(&sc0, 0, sizeof(sc0));
    for (int sp = 0; sp < 2; ++sp) {
        const int64_t n = init ? init[sp].n : 0;
        if (n > h->cap[sp])
            return fail(h, PIC_ECAPACITY, "species %d: %lld initial particles > capacity %lld", sp,
                        (long long)n, (long long)h->cap[sp]);
        uint32_t mx = 0;
        if (n > 0) {
            const pic_species_host &I = init[sp];
            if (!I.r || !I.z || !I.vr || !I.vt || !I.vz || !I.id)
                return fail(h, PIC_EINVAL, "species %d: initial arrays missing", sp);
            for (int64_t k = 0; k < n; ++k) {
                if (!(I.r[k] >= 0.0 && I.r[k] < c.lr && I.z[k] >= 0.0 && I.z[k] < c.lz))
                    return fail(h, PIC_EINVAL, "species %d particle %lld outside the domain", sp,
                                (long long)k);
                mx = std::max(mx, I.id[k] + 1u);
            }
            // upload in chunks through the second buffer
            const Buf &stage = h->buf[sp][1];
            const int64_t stage_bytes = h->cap[sp] * (8 + 5 * (int64_t)sizeof(T));
            const int64_t chunk = std::max<int64_t>(1, stage_bytes / 48);
            double *dr = (double *)stage.key;
            for (int64_t o = 0; o < n; o += chunk) {
                const int64_t m = std::min(chunk, n - o);
                double *a0 = dr, *a1 = dr + m, *a2 = dr + 2 * m, *a3 = dr + 3 * m, *a4 = dr + 4 * m;
                uint32_t *ai = (uint32_t *)(dr + 5 * m);
                HIPCHECK(h, hipMemcpy(a0, I.r + o, m * 8, hipMemcpyHostToDevice));
                HIPCHECK(h, hipMemcpy(a1, I.z + o, m * 8, hipMemcpyHostToDevice));
                HIPCHECK(h, hipMemcpy(a2, I.vr + o, m * 8, hipMemcpyHostToDevice));
                HIPCHECK(h, hipMemcpy(a3, I.vt + o, m * 8, hipMemcpyHostToDevice));
                HIPCHECK(h, hipMemcpy(a4, I.vz + o, m * 8, hipMemcpyHostToDevice));
                HIPCHECK(h, hipMemcpy(ai, I.id + o, m * 4, hipMemcpyHostToDevice));
                launch_load<T>(species_dev<T>(h->buf[sp][0]), o, a0, a1, a2, a3, a4, ai, m, c.nr,
                               c.nz, c.lr / c.nr, c.lz / c.nz, s);
                HIPCHECK(h, hipStreamSynchronize(s));
            }
        }
        sc0.count[sp] = n;
        sc0.next_id[sp] = mx;
        h->host_count[sp] = n;
    }
    sc0.cap_c = 0.0;
    HIPCHECK(h, hipMemcpy(h->sc, &sc0, sizeof(DevScalars), hipMemcpyHostToDevice));
    h->cur[0] = h->cur[1] = 0;
    sort_all<T>(h);
    const int64_t nodes = (int64_t)(c.nr + 1) * (c.nz + 1);
    // phi_L: cathode at 1 V, no charge
    launch_begin_step(h->sc, h->q[0], h->q[1], nodes, (int)sizeof(T), s);
    launch_zero(h->f.phi_l, nodes * 8, s);
    const int init_mode = (h->pmode == PIC_DIRECT) ? PIC_DIRECT : PIC_MGCG;
    st = solve<T>(h, h->f.phi_l, (const T *)h->q[0], (const T *)h->q[1], 1.0, nullptr, init_mode);
    if (st != PIC_OK) return st;
    // capacitance C = sum over cathode nodes of (K phi_L)
    {
        std::vector<double> pl(nodes), ce(nodes), cn(nodes);
        HIPCHECK(h, hipMemcpy(pl.data(), h->f.phi_l, nodes * 8, hipMemcpyDeviceToHost));
        host_couplings(c.nr, c.nz, c.lr, c.lz, eps0(), ce.data(), cn.data());
        double cap = 0.0;
        const int ld = c.nr + 1;
        for (int i = 0; i <= c.nr; ++i) {
            if (host_node_kind(c.nr, c.nz, c.lr, c.cathode_rmax, i, 0) != 1) continue;
            double fl = 0.0;
            if (i < c.nr) fl += ce[i] * (pl[i] - pl[i + 1]);
            if (i > 0) fl += ce[i - 1] * (pl[i] - pl[i - 1]);
            fl += cn[i] * (pl[i] - pl[i + ld]);
            cap += fl;
        }
        HIPCHECK(h, hipMemcpy(&h->sc->cap_c, &cap, 8, hipMemcpyHostToDevice));
    }
    // initial deposit, phi0, circuit state at V0, gather fields
    launch_begin_step(h->sc, h->q[0], h->q[1], nodes, (int)sizeof(T), s);
    launch_push_h<T>(h, 1);
    if (c.deposit_fixed) {
        const double qw64[2] = {c.q[0] * c.w[0], c.q[1] * c.w[1]};
        launch_q_from_fixed(h->q[0], h->q[1], nodes, qw64, s);
    }
    launch_zero(h->f.phi0, nodes * 8, s);
    if (c.field_solve) {
        st = solve<T>(h, h->f.phi0, (const T *)h->q[0], (const T *)h->q[1], 0.0, nullptr,
                      init_mode);
        if (st != PIC_OK) return st;
    }
    launch_extrapolate(h->f, 1, s);
    const double v0 = (c.circuit == PIC_RESISTOR) ? c.v_ext : c.v_fixed;
    launch_circuit<T>(h->f, (const T *)h->q[0], (const T *)h->q[1], h->sc, PIC_FIXED_V, v0, 0.0,
                      1.0, c.dt, 0.0, s);
    launch_field_prep<T>(h->f, (typename Vec4<T>::type *)h->node, h->sc, c.scheme, 0, s);
    // clear the tallies of the deposit pass
    launch_begin_step(h->sc, h->q[0], h->q[1], 0, (int)sizeof(T), s);
    HIPCHECK(h, hipStreamSynchronize(s));
    h->steps_since_sort = 0;
    return check_flags(h);
}

// ---- ensembles ---------------------------------------------------------------
}  // namespace

struct pic_ensemble {
    std::vector<pic_handle *> runs;
    hipStream_t s0 = nullptr;
    bool own_s0 = false;
    RunStatus *status = nullptr;        // pinned host memory, one per run
    RunStatus *status_dev = nullptr;    // its device address
    std::vector<BatchPlan> plans;       // batches of at most MAX_BATCH runs
    struct G {
        int sort, cur0, cur1;
        hipGraphExec_t exec;
    };
    std::vector<G> graphs;
    hipGraphExec_t pass_exec = nullptr; // a further solve pass (runs not yet converged)
    std::vector<int64_t> captured;      // particles per run when the graphs were captured
    std::string err;
};

namespace {

pic_status efail(pic_ensemble *e, pic_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    if (e) e->err = buf;
    else g_init_error = buf;
    return st;
}

#define EHIPCHECK(e, call)                                                                  \
    do {                                                                                    \
        hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess)                                                               \
            return efail((e), PIC_EHIP, "%s failed: %s", #call, hipGetErrorString(e_));     \
    } while (0)

void drop_ensemble_graphs(pic_ensemble *e)
{
    for (auto &g : e->graphs) (void)hipGraphExecDestroy(g.exec);
    e->graphs.clear();
    if (e->pass_exec) (void)hipGraphExecDestroy(e->pass_exec);
    e->pass_exec = nullptr;
}

// A run's RunParticles for the four pairs of current particle buffers, into
// its workspace.
template <typename T>
bool upload_run_particles(pic_handle *h)
{
    const int cur0 = h->cur[0], cur1 = h->cur[1];
    bool up = true;
    for (int k = 0; k < 4; ++k) {
        h->cur[0] = k & 1;
        h->cur[1] = k >> 1;
        RunParticles<T> D;
        memset(&D, 0, sizeof(D));
        D.push = push_params<T>(h, 0);
        D.ev = event_params<T>(h);
        D.ch = child_params<T>(h);
        for (int sp = 0; sp < 2; ++sp) {
            SortJob<T> &J = D.sort[sp];
            J.src = species_dev<T>(h->buf[sp][h->cur[sp]]);
            J.dst = species_dev<T>(h->buf[sp][1 - h->cur[sp]]);
            J.sc = h->sc;
            J.hist = h->hist;
            J.block_sums = h->block_sums;
            J.nr = h->cfg.nr;
            J.nbins = h->cfg.nr * h->cfg.nz;
        }
        up &= hipMemcpy(h->part_desc + k * PART_DESC_BYTES, &D, sizeof(D),
                        hipMemcpyHostToDevice) == hipSuccess;
    }
    h->cur[0] = cur0;
    h->cur[1] = cur1;
    return up;
}

// Cell sort of both species of the runs of batch b, from their current
// buffers (the descriptor of the runs' current pair).
template <typename T>
void sort_b(pic_ensemble *e, size_t b)
{
    const size_t r0 = b * MAX_BATCH;
    const size_t r1 = std::min(e->runs.size(), r0 + MAX_BATCH);
    const int n = (int)(r1 - r0);
    SortBatch<T> B;
    memset(&B, 0, sizeof(B));
    B.nruns = n;
    int64_t cap[2][MAX_BATCH];
    for (int k = 0; k < n; ++k) {
        pic_handle *h = e->runs[r0 + k];
        const RunParticles<T> *d =
            (const RunParticles<T> *)(h->part_desc + (h->cur[0] + 2 * h->cur[1]) * PART_DESC_BYTES);
        B.job[k] = d->sort;
        B.nbins[k] = h->cfg.nr * h->cfg.nz;
        cap[0][k] = h->cap[0];
        cap[1][k] = h->cap[1];
    }
    for (int sp = 0; sp < 2; ++sp) {
        B.species = sp;
        launch_sort_b<T>(B, cap[sp], e->s0);
    }
}

// Particle phase of the runs of batch b of an ensemble, one launch per
// kernel (begin, push, events, children, finalize), each block reading its
// run's descriptor for the run's current particle buffers.  A batch that
// mixes schemes pushes run by run.
template <typename T>
void particle_phase_b(pic_ensemble *e, size_t b)
{
    const size_t r0 = b * MAX_BATCH;
    const size_t r1 = std::min(e->runs.size(), r0 + MAX_BATCH);
    const int n = (int)(r1 - r0);
    PartBatch<T> Bb, Bp, Be, Bc;
    for (PartBatch<T> *B : {&Bb, &Bp, &Be, &Bc}) memset(B, 0, sizeof(*B));
    int ob = 0, op = 0, oe = 0, oc = 0;
    bool one_scheme = true;
    for (int k = 0; k < n; ++k) {
        pic_handle *h = e->runs[r0 + k];
        one_scheme &= h->cfg.scheme == e->runs[r0]->cfg.scheme;
        const RunParticles<T> *d =
            (const RunParticles<T> *)(h->part_desc + (h->cur[0] + 2 * h->cur[1]) * PART_DESC_BYTES);
        Bb.p[k] = d;
        Bb.off[k] = ob;
        ob += begin_b_blocks((int64_t)(h->cfg.nr + 1) * (h->cfg.nz + 1), (int)sizeof(T));
        Bp.off[k] = op;
        int be, nb;
        push_grid(h, &be, &nb);
        Bp.aux[k] = be;
        op += nb;
        Be.off[k] = oe;
        oe += EVENTS_B_BLOCKS;
        Bc.off[k] = oc;
        oc += children_b_blocks(h->child_cap);
    }
    Bb.off[n] = ob;
    Bb.nruns = n;
    for (PartBatch<T> *B : {&Bp, &Be, &Bc}) {
        for (int k = 0; k < n; ++k) B->p[k] = Bb.p[k];
        B->nruns = n;
    }
    Bp.off[n] = op;
    Be.off[n] = oe;
    Bc.off[n] = oc;
    launch_begin_b<T>(Bb, e->s0);
    if (one_scheme) {
        launch_push_b<T>(Bp, e->runs[r0]->cfg.scheme, e->s0);
    } else {
        for (size_t r = r0; r < r1; ++r) {
            pic_handle *h = e->runs[r];
            hipStream_t saved = h->stream;
            h->stream = e->s0;
            launch_push_h<T>(h, 0);
            h->stream = saved;
        }
    }
    launch_events_b<T>(Be, e->s0);
    launch_children_b<T>(Bc, e->s0);
    launch_finalize_b<T>(Bb, e->s0);
}

// One device-gated multigrid-PCG pass of n iterations for the runs of batch
// b that have not converged, then circuit and gather fields of the runs
// converged and not yet finished (the status copy marks them finished).
void enqueue_pass_b(pic_ensemble *e, size_t b, int n, hipStream_t s)
{
    const BatchPlan &P = e->plans[b];
    if (batch_fused_cg(P)) {
        // CG vector work in the finest level's V-cycle kernels (the cast
        // clears the pass's slotted dots)
        launch_nodes_b(P, BATCH_CAST_SCALE_CG, s, n);
        for (int k = 0; k < n; ++k) launch_mg_vcycle_cg_b(P, k, s);
        launch_cg_update_last_b(P, n - 1, s);
    } else {
        launch_nodes_b(P, BATCH_CAST_SCALE, s);
        launch_scalars_b(P, BATCH_ZERO_PCG_GATED, 0, s);
        launch_mg_vcycle_b(P, 0, s);
        for (int k = 0; k < n; ++k) {
            launch_cg_matvec_b(P, k, s);
            launch_cg_update_b(P, k, s);
            if (k + 1 < n) launch_mg_vcycle_b(P, k + 1, s);
        }
    }
    launch_nodes_b(P, BATCH_UPDATE64, s);
    launch_scalars_b(P, BATCH_ZERO_RES_GATED, 0, s);
    launch_residual64_b(P, 1, s);
    launch_scalars_b(P, BATCH_SOLVE_GATE, n, s);
    launch_circuit_b(P, s);
    launch_nodes_b(P, BATCH_FIELD_PREP, s);
    launch_status_b(P, e->status_dev + b * MAX_BATCH, s);
}

// The further pass of an ensemble step, launched only when a run has not
// converged after the step's first pass.
pic_status capture_pass(pic_ensemble *e, int n)
{
    EHIPCHECK(e, hipStreamBeginCapture(e->s0, hipStreamCaptureModeThreadLocal));
    for (size_t b = 0; b < e->plans.size(); ++b) enqueue_pass_b(e, b, n, e->s0);
    hipGraph_t graph;
    const hipError_t ec = hipStreamEndCapture(e->s0, &graph);
    if (ec != hipSuccess)
        return efail(e, PIC_EHIP, "capture of the ensemble pass failed: %s", hipGetErrorString(ec));
    const hipError_t ei = hipGraphInstantiate(&e->pass_exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ei != hipSuccess) {
        e->pass_exec = nullptr;
        return efail(e, PIC_EHIP, "graph instantiation failed: %s", hipGetErrorString(ei));
    }
    return PIC_OK;
}

// Capture one step of every run: for each batch of up to MAX_BATCH runs one
// launch per kernel (in a sort step the cell sort of each species first),
// the batched field update and a status copy per run.
pic_status capture_ensemble(pic_ensemble *e, bool do_sort, hipGraphExec_t *out)
{
    std::vector<int> cur0, cur1, since;
    for (pic_handle *h : e->runs) {
        cur0.push_back(h->cur[0]);
        cur1.push_back(h->cur[1]);
        since.push_back(h->steps_since_sort);
    }
    // pass plan of the batched solve, from the runs' measured convergence
    double rho = 0.0, rel0 = 0.0, rtol = 1.0;
    for (pic_handle *h : e->runs) {
        rho = std::max(rho, h->rho);
        rel0 = std::max(rel0, h->rel0_est);
        rtol = std::min(rtol, h->cfg.poisson_rtol);
    }
    auto iters = [&](double target) {
        const int n = (int)std::ceil(std::log(target) / std::log(rho));
        return std::max(1, std::min(n, 64));
    };
    const int plan[2] = {iters(std::max(0.5 * rtol / rel0, 1e-6)), iters(1e-6)};
    if (!e->pass_exec) {
        pic_status st = capture_pass(e, plan[1]);
        if (st != PIC_OK) return st;
    }
    EHIPCHECK(e, hipStreamBeginCapture(e->s0, hipStreamCaptureModeThreadLocal));
    // the sorts of a sort step: each species of every run of a batch, one
    // launch per kernel; then every run's current buffers flip
    if (do_sort) {
        for (size_t b = 0; b < e->plans.size(); ++b) {
            if (e->runs[0]->prec == PIC_F64) sort_b<double>(e, b);
            else sort_b<float>(e, b);
        }
        for (pic_handle *h : e->runs) {
            h->cur[0] = 1 - h->cur[0];
            h->cur[1] = 1 - h->cur[1];
            h->steps_since_sort = 0;
        }
    }
    // particle phase of every run: one launch per kernel for a batch of runs
    for (size_t b = 0; b < e->plans.size(); ++b) {
        if (e->runs[0]->prec == PIC_F64) particle_phase_b<double>(e, b);
        else particle_phase_b<float>(e, b);
    }
    // field update of every run, batched: extrapolated warm start, FP64
    // residual, the first device-gated multigrid-PCG pass, then circuit,
    // gather fields and status of the runs it converged
    hipStream_t s = e->s0;
    for (size_t b = 0; b < e->plans.size(); ++b) {
        const BatchPlan &P = e->plans[b];
        launch_nodes_b(P, BATCH_EXTRAPOLATE, s);
        launch_nodes_b(P, BATCH_SET_DIRICHLET, s);
        launch_scalars_b(P, BATCH_ZERO_RES, 0, s);
        launch_residual64_b(P, 0, s);
        launch_scalars_b(P, BATCH_SOLVE_INIT, 0, s);
        launch_nodes_b(P, BATCH_ZERO_IF_EMPTY, s);
        enqueue_pass_b(e, b, plan[0], s);
    }
    hipGraph_t graph;
    const hipError_t ec = hipStreamEndCapture(e->s0, &graph);
    // the capture ran nothing: restore the host-side particle-buffer state
    for (size_t r = 0; r < e->runs.size(); ++r) {
        e->runs[r]->cur[0] = cur0[r];
        e->runs[r]->cur[1] = cur1[r];
        e->runs[r]->steps_since_sort = since[r];
    }
    if (ec != hipSuccess)
        return efail(e, PIC_EHIP, "capture of the ensemble step failed: %s", hipGetErrorString(ec));
    const hipError_t ei = hipGraphInstantiate(out, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ei != hipSuccess)
        return efail(e, PIC_EHIP, "graph instantiation failed: %s", hipGetErrorString(ei));
    return PIC_OK;
}

pic_status ensemble_step(pic_ensemble *e)
{
    pic_handle *h0 = e->runs[0];
    const bool do_sort = h0->steps_since_sort >= h0->cfg.sort_every;
    hipGraphExec_t exec = nullptr;
    for (auto &g : e->graphs)
        if (g.sort == (int)do_sort && g.cur0 == h0->cur[0] && g.cur1 == h0->cur[1]) exec = g.exec;
    if (!exec) {
        pic_status st = capture_ensemble(e, do_sort, &exec);
        if (st != PIC_OK) return st;
        e->graphs.push_back({(int)do_sort, h0->cur[0], h0->cur[1], exec});
        e->captured.clear();
        for (pic_handle *h : e->runs) e->captured.push_back(h->host_count[0] + h->host_count[1]);
    }
    // work a run's own stream still holds goes first
    for (pic_handle *h : e->runs) EHIPCHECK(e, hipStreamSynchronize(h->stream));
    EHIPCHECK(e, hipGraphLaunch(exec, e->s0));
    EHIPCHECK(e, hipStreamSynchronize(e->s0));
    // up to two further passes while some run has not converged
    for (int p = 1; p < 3; ++p) {
        bool open = false;
        for (size_t r = 0; r < e->runs.size(); ++r)
            open |= e->status[(r / MAX_BATCH) * MAX_BATCH + r % MAX_BATCH].solve_done == 0;
        if (!open) break;
        EHIPCHECK(e, hipGraphLaunch(e->pass_exec, e->s0));
        EHIPCHECK(e, hipStreamSynchronize(e->s0));
    }
    bool drift = false;
    for (size_t r = 0; r < e->runs.size(); ++r) {
        pic_handle *h = e->runs[r];
        const RunStatus &S = e->status[(r / MAX_BATCH) * MAX_BATCH + r % MAX_BATCH];
        if (do_sort) {
            h->cur[0] = 1 - h->cur[0];
            h->cur[1] = 1 - h->cur[1];
            h->steps_since_sort = 0;
        }
        h->steps_since_sort++;
        h->host_count[0] = S.count[0];
        h->host_count[1] = S.count[1];
        h->host_flags = S.flags;
        pic_poisson_stats P = {};
        P.iterations = S.solve_iters;
        P.outer = S.solve_passes;
        P.rel_res = S.bb > 0.0 ? std::sqrt(S.rr / S.bb) : 0.0;
        P.converged = S.solve_done;
        h->last = P;
        if (S.flags & (FLAG_CAPACITY | FLAG_CHILD_OVERFLOW))
            return efail(e, PIC_ECAPACITY, "run %zu: particle capacity exceeded (flags %d)", r,
                         S.flags);
        if (h->cfg.field_solve && !S.solve_done)
            return efail(e, PIC_ENOCONV, "run %zu: field solve stopped at relative residual %.3e",
                         r, P.rel_res);
        const int64_t n = S.count[0] + S.count[1], c = e->captured[r];
        if (std::llabs(n - c) > std::max<int64_t>(c / 5, 1024)) drift = true;
    }
    // the push launches split their blocks by the counts seen at capture
    if (drift) drop_ensemble_graphs(e);
    return PIC_OK;
}

}  // namespace

// ---- scratch of pic_poisson_static ------------------------------------------
// A file-scope device array: each GPU the library runs on holds its own copy
// until the process ends.  Host code never passes the array's name to a
// kernel (on the host it is a stand-in, not a device address): the device
// address of each GPU's copy comes from hipGetSymbolAddress, taken once per
// device with that device current, and only that pointer is used.
constexpr int64_t STATIC_SCRATCH_BYTES = 32ll << 20;
constexpr int MAX_DEVICES = 64;
static __device__ __align__(256) char scratch[STATIC_SCRATCH_BYTES];

namespace {

std::mutex g_scratch_mu;
char *g_scratch_dev[MAX_DEVICES] = {};

// Device address of the current device's scratch (nullptr on failure).
hipError_t scratch_of_device(int dev, char **out)
{
    *out = nullptr;
    if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_dev[dev] = (char *)ptr;
    }
    *out = g_scratch_dev[dev];
    return hipSuccess;
}

// Bytes of scratch a direct solve of the handle's grid takes: scalar block
// (the residual norms' slots), the FP64 residual, the transform buffers.
int64_t static_scratch_bytes(const pic_handle *h)
{
    const int64_t nodes = (int64_t)(h->cfg.nr + 1) * (h->cfg.nz + 1);
    const int64_t Mp = fs_pad(h->cfg.nz - 1), Np = fs_pad(h->cfg.nr);
    auto up = [](int64_t b) { return (b + 255) & ~(int64_t)255; };
    return up(sizeof(DevScalars)) + up(nodes * 8) + 2 * up(Mp * Np * 8);
}

template <typename T>
pic_status plasma_typed(pic_handle *h, double r0, double r1, pic_plasma_out *out,
                        double *maps_host)
{
    const pic_config &c = h->cfg;
    const int64_t ncell = (int64_t)c.nr * c.nz;
    hipStream_t s = h->stream;
    launch_zero(h->pd.mom[0], 5 * ncell * 8, s);
    launch_zero(h->pd.mom[1], 5 * ncell * 8, s);
    for (int sp = 0; sp < 2; ++sp)
        launch_cell_moments<T>(species_dev<T>(h->buf[sp][h->cur[sp]]), h->host_count[sp], c.nr,
                               c.nz, h->pd.mom[sp], s);
    PlasmaArgs A;
    A.nr = c.nr;
    A.nz = c.nz;
    A.dr = c.lr / c.nr;
    A.dz = c.lz / c.nz;
    A.w[0] = c.w[0];
    A.w[1] = c.w[1];
    A.m_e = c.m[0];
    // band cells: centre (i + 1/2) dr in [r0, r1)
    A.ib0 = c.nr;
    A.ib1 = c.nr;
    for (int i = c.nr - 1; i >= 0; --i) {
        const double rc = (i + 0.5) * A.dr;
        if (rc >= r1) A.ib1 = i;
        if (rc >= r0) A.ib0 = i;
    }
    if (A.ib1 < A.ib0) A.ib1 = A.ib0;
    launch_plasma(h->pd, A, h->f.phi, s);
    PlasmaOut o;
    HIPCHECK(h, hipMemcpyAsync(&o, h->pd.out, sizeof(o), hipMemcpyDeviceToHost, s));
    if (maps_host)
        HIPCHECK(h, hipMemcpyAsync(maps_host, h->pd.maps, 4 * ncell * 8, hipMemcpyDeviceToHost, s));
    HIPCHECK(h, hipStreamSynchronize(s));
    out->z_sheath = o.z_sheath;
    out->z_bulk = o.z_bulk;
    for (int r = 0; r < 3; ++r) {
        out->te_region[r] = o.te_region[r];
        out->n_region[r] = (int64_t)o.n_region[r];
    }
    out->lambda_d_peak = o.lambda_d_peak;
    out->n_e_peak = o.n_e_peak;
    out->te_peak = o.te_peak;
    out->peak_cell[0] = o.peak_i;
    out->peak_cell[1] = o.peak_j;
    out->band_cells[0] = A.ib0;
    out->band_cells[1] = A.ib1;
    return PIC_OK;
}

template <typename T>
pic_status reweight_typed(pic_handle *h, int32_t k)
{
    pic_config &c = h->cfg;
    for (int s = 0; s < 2; ++s)
        launch_reweight<T>(species_dev<T>(h->buf[s][h->cur[s]]), h->host_count[s], (uint32_t)k,
                           h->stream);
    sort_all<T>(h);
    c.w[0] *= k;
    c.w[1] *= k;
    h->t_see[0] = host_see_threshold(c, 0);
    h->t_see[1] = host_see_threshold(c, 1);
    PushCold<T> C = push_cold<T>(h);
    HIPCHECK(h, hipMemcpyAsync(h->cold, &C, sizeof(C), hipMemcpyHostToDevice, h->stream));
    return check_flags(h);
}

}  // namespace

extern "C" {

pic_status pic_query_workspace(const pic_config *cfg, int64_t *bytes)
{
    pic_status st = validate(cfg, nullptr);
    if (st != PIC_OK) return st;
    if (!bytes) return fail(nullptr, PIC_EINVAL, "bytes is NULL");
    *bytes = layout(*cfg, nullptr, nullptr);
    return PIC_OK;
}

pic_status pic_init(const pic_config *cfg, void *workspace_dev, int64_t workspace_bytes,
                    void *stream, const pic_species_host *init, pic_handle **out)
{
    if (!out) return fail(nullptr, PIC_EINVAL, "out is NULL");
    *out = nullptr;
    pic_status st = validate(cfg, nullptr);
    if (st != PIC_OK) return st;
    const int64_t need = layout(*cfg, nullptr, nullptr);
    if (!workspace_dev || workspace_bytes < need)
        return fail(nullptr, PIC_EINVAL, "workspace of %lld bytes < %lld needed",
                    (long long)workspace_bytes, (long long)need);
    if (((uintptr_t)workspace_dev & 255) != 0)
        return fail(nullptr, PIC_EINVAL, "workspace must be 256-byte aligned");
    pic_handle *h = new pic_handle();
    h->cfg = *cfg;
    h->stream = (hipStream_t)stream;
    if (hipGetDevice(&h->device) != hipSuccess) h->device = 0;
    h->ws = (char *)workspace_dev;
    h->ws_bytes = workspace_bytes;
    h->prec = cfg->precision;
    h->ts = (cfg->precision == PIC_F64) ? 8 : 4;
    h->cap[0] = cfg->capacity[0];
    h->cap[1] = cfg->capacity[1];
    h->pmode = cfg->poisson_mode;
    layout(*cfg, h->ws, h);
    if (hipHostMalloc((void **)&h->pinned, PINNED_BYTES) != hipSuccess) {
        h->pinned = nullptr;
        st = fail(h, PIC_EHIP, "cannot allocate %zu bytes of pinned host memory", PINNED_BYTES);
    } else if (hipEventCreateWithFlags(&h->rb_done, hipEventDisableTiming) != hipSuccess) {
        h->rb_done = nullptr;
        st = fail(h, PIC_EHIP, "cannot create the readback event");
    } else {
        st = (h->prec == PIC_F64) ? init_typed<double>(h, init) : init_typed<float>(h, init);
    }
    // the host arrays of the config are not kept
    h->cfg.sigma = nullptr;
    h->cfg.b_r = h->cfg.b_z = nullptr;
    if (st != PIC_OK) {
        g_init_error = h->err;
        (void)hipStreamSynchronize(h->stream);
        if (h->pinned) (void)hipHostFree(h->pinned);
        if (h->rb_done) (void)hipEventDestroy(h->rb_done);
        delete h;
        return st;
    }
    *out = h;
    return PIC_OK;
}

pic_status pic_step(pic_handle *h, int32_t nsteps)
{
    if (!h) return fail(nullptr, PIC_EINVAL, "handle is NULL");
    if (nsteps < 0) return fail(h, PIC_EINVAL, "nsteps < 0");
    for (int k = 0; k < nsteps; ++k) {
        pic_status st = (h->prec == PIC_F64) ? step_one<double>(h) : step_one<float>(h);
        if (st != PIC_OK) return st;
    }
    // with the direct solve no step synchronized: capacity, overflow and
    // solve flags of all the call's steps are read here, once
    if (nsteps > 0 && h->cfg.field_solve && h->pmode == PIC_DIRECT) return check_flags(h);
    return PIC_OK;
}

pic_status pic_poisson(pic_handle *h, const double *q_dev, double v_cathode, double *phi_dev,
                       pic_poisson_stats *stats)
{
    if (!h) return fail(nullptr, PIC_EINVAL, "handle is NULL");
    if (!q_dev || !phi_dev) return fail(h, PIC_EINVAL, "q_dev and phi_dev are required");
    hipEvent_t ev[2];
    timer_begin(h, ev, 3);
    pic_status st = solve<double>(h, phi_dev, q_dev, (const double *)nullptr, v_cathode, stats,
                                  h->pmode);
    timer_end(h, 3, ev);
    return st;
}

pic_status pic_poisson_static(pic_handle *h, const double *q_dev, double v_cathode,
                              double *phi_dev, pic_poisson_stats *stats)
{
    if (!h) return fail(nullptr, PIC_EINVAL, "handle is NULL");
    if (!q_dev || !phi_dev) return fail(h, PIC_EINVAL, "q_dev and phi_dev are required");
    if (!h->fs_on)
        return fail(h, PIC_ESTATE, "pic_poisson_static needs a handle created with PIC_DIRECT");
    const int64_t need = static_scratch_bytes(h);
    if (need > STATIC_SCRATCH_BYTES)
        return fail(h, PIC_EINVAL,
                    "grid %d x %d needs %lld bytes of scratch, above the %lld of "
                    "pic_poisson_static",
                    h->cfg.nr, h->cfg.nz, (long long)need, (long long)STATIC_SCRATCH_BYTES);
    int dev = -1;
    HIPCHECK(h, hipGetDevice(&dev));
    if (dev != h->device)
        return fail(h, PIC_EINVAL, "device %d is current; the handle lives on device %d", dev,
                    h->device);
    char *base = nullptr;
    HIPCHECK(h, scratch_of_device(dev, &base));
    // the solve's temporaries in the scratch; the handle gives the operator
    // and the transform tables
    auto up = [](int64_t b) { return (b + 255) & ~(int64_t)255; };
    const int64_t nodes = (int64_t)(h->cfg.nr + 1) * (h->cfg.nz + 1);
    const int64_t Mp = fs_pad(h->cfg.nz - 1), Np = fs_pad(h->cfg.nr);
    DevScalars *ssc = (DevScalars *)base;
    FieldDev f = h->f;
    f.r64 = (double *)(base + up(sizeof(DevScalars)));
    FastSolve F = h->fs;
    F.b = (double *)((char *)f.r64 + up(nodes * 8));
    F.bh = (double *)((char *)F.b + up(Mp * Np * 8));
    hipStream_t s = h->stream;
    const double rtol = h->cfg.poisson_rtol;
    pic_poisson_stats S = {};
    // Dirichlet values and cleared norms, FP64 residual, then corrections
    // (as pic_poisson with PIC_DIRECT)
    launch_solve_prep(f, phi_dev, false, v_cathode, ssc, s);
    launch_residual64<double>(f, phi_dev, q_dev, nullptr, ssc, s, false);
    double *pin = (double *)h->pinned;
    for (;;) {
        launch_fast_solve(F, f, phi_dev, ssc, s);
        launch_residual64<double>(f, phi_dev, q_dev, nullptr, ssc, s, false);
        S.outer++;
        HIPCHECK(h, hipMemcpyAsync(pin, ssc->res_slots, RES_SLOT_WORDS * sizeof(double),
                                   hipMemcpyDeviceToHost, s));
        HIPCHECK(h, hipStreamSynchronize(s));
        double rr = 0.0, bb = 0.0;
        for (int k = 0; k < ACC_SLOTS; ++k) {
            rr += pin[k * ACC_STRIDE];
            bb += pin[(ACC_SLOTS + k) * ACC_STRIDE];
        }
        S.rel_res = bb > 0.0 ? std::sqrt(rr / bb) : 0.0;
        S.converged = (std::isfinite(S.rel_res) && S.rel_res <= rtol) ? 1 : 0;
        if (S.converged || !std::isfinite(S.rel_res) || S.outer == 3) break;
    }
    if (stats) *stats = S;
    if (!std::isfinite(S.rel_res)) return fail(h, PIC_ENAN, "non-finite residual in the field solve");
    if (!S.converged)
        return fail(h, PIC_ENOCONV, "direct field solve left relative residual %.3e (target %.1e)",
                    S.rel_res, rtol);
    return PIC_OK;
}

pic_status pic_diag(pic_handle *h, pic_diag_out *out)
{
    if (!h || !out) return fail(h, PIC_EINVAL, "NULL argument");
    const pic_config &c = h->cfg;
    memset(out, 0, sizeof(*out));
    launch_zero(h->live, 16, h->stream);
    for (int s = 0; s < 2; ++s)
        launch_count_live(live_key_words(h, s), h->sc, s, h->live + s, h->stream);
    if (h->prec == PIC_F64)
        launch_diag_grid<double>(h->f, (const double *)h->q[0], (const double *)h->q[1], c.q[0],
                                 c.q[1], h->diag_partials, h->diag_blocks, h->stream);
    else
        launch_diag_grid<float>(h->f, (const float *)h->q[0], (const float *)h->q[1], c.q[0],
                                c.q[1], h->diag_partials, h->diag_blocks, h->stream);
    std::vector<double> part((size_t)h->diag_blocks * 6);
    unsigned long long live[2];
    HIPCHECK(h, hipMemcpyAsync(part.data(), h->diag_partials, part.size() * 8,
                               hipMemcpyDeviceToHost, h->stream));
    HIPCHECK(h, hipMemcpyAsync(live, h->live, 16, hipMemcpyDeviceToHost, h->stream));
    DevScalars sc;
    pic_status st = read_scalars(h, &sc);
    if (st != PIC_OK) return st;
    double s0 = 0, s1 = 0, m0 = -1e300, m1 = -1e300, mp = -1e300, w = 0;
    for (int b = 0; b < h->diag_blocks; ++b) {
        s0 += part[b * 6 + 0];
        s1 += part[b * 6 + 1];
        m0 = std::max(m0, part[b * 6 + 2]);
        m1 = std::max(m1, part[b * 6 + 3]);
        mp = std::max(mp, part[b * 6 + 4]);
        w += part[b * 6 + 5];
    }
    out->step = sc.step;
    out->time = sc.step * c.dt;
    for (int s = 0; s < 2; ++s) {
        out->count[s] = (int64_t)live[s];
        out->q_expect[s] = c.q[s] * c.w[s] * (double)live[s];
        out->ke[s] = sc.ke[s];
        out->pz[s] = sc.pz[s];
        for (int k = 0; k < 5; ++k) out->n_abs[s][k] = (int64_t)sc.n_abs[s][k];
    }
    out->q_dep[0] = s0;
    out->q_dep[1] = s1;
    out->n_peak[0] = m0;
    out->n_peak[1] = m1;
    out->phi_max = mp;
    out->w_field = w;
    out->dq_conv = sc.dq_conv;
    out->i_cathode = sc.dq_conv / c.dt;
    out->vc = sc.vc;
    out->qc = sc.qc;
    out->cap_c = sc.cap_c;
    out->n_cand = (int64_t)sc.n_cand;
    for (int k = 0; k < 4; ++k) out->n_coll[k] = (int64_t)sc.n_coll[k];
    out->n_see = (int64_t)sc.n_see;
    out->n_see_e = (int64_t)sc.n_see_e;
    out->deposit_fallback = (int64_t)sc.deposit_fallback;
    out->poisson = h->last;
    if (h->last.converged == -1) {
        // a step's direct solve: its FP64 residual norms are still on the device
        double rr = 0.0, bb = 0.0;
        for (int k = 0; k < ACC_SLOTS; ++k) {
            rr += sc.res_slots[k * ACC_STRIDE];
            bb += sc.res_slots[(ACC_SLOTS + k) * ACC_STRIDE];
        }
        out->poisson.rel_res = bb > 0.0 ? std::sqrt(rr / bb) : 0.0;
        out->poisson.converged = out->poisson.rel_res <= c.poisson_rtol ? 1 : 0;
    }
    out->flags = sc.flags;
    if (!std::isfinite(w) || !std::isfinite(sc.ke[0]) || !std::isfinite(sc.ke[1]))
        out->flags |= FLAG_NAN;
    return PIC_OK;
}

pic_status pic_particles(pic_handle *h, int32_t species, pic_particle_view *out)
{
    if (!h || !out || species < 0 || species > 1) return fail(h, PIC_EINVAL, "bad argument");
    int64_t cnt;
    HIPCHECK(h, hipMemcpyAsync(&cnt, &h->sc->count[species], 8, hipMemcpyDeviceToHost, h->stream));
    HIPCHECK(h, hipStreamSynchronize(h->stream));
    const Buf &b = h->buf[species][h->cur[species]];
    out->key_dev = h->prec == PIC_F64 ? b.key : nullptr;
    out->pos_bits = h->prec == PIC_F64 ? 0 : POS_BITS;
    out->fr_dev = b.fr;
    out->fz_dev = b.fz;
    out->vr_dev = b.vr;
    out->vt_dev = b.vt;
    out->vz_dev = b.vz;
    out->id_dev = b.id;
    out->count = cnt;
    out->capacity = h->cap[species];
    out->precision = h->prec;
    return PIC_OK;
}

pic_status pic_fields(pic_handle *h, pic_field_view *out)
{
    if (!h || !out) return fail(h, PIC_EINVAL, "bad argument");
    out->phi_dev = h->f.phi;
    out->phi0_dev = h->f.phi0;
    out->phi_l_dev = h->f.phi_l;
    out->q_dev[0] = h->q[0];
    out->q_dev[1] = h->q[1];
    out->nodes = (int64_t)(h->cfg.nr + 1) * (h->cfg.nz + 1);
    out->q_precision = h->prec;
    out->phi0_prev_dev = h->f.phi0_prev;
    return PIC_OK;
}

pic_status pic_set_phi(pic_handle *h, const double *phi)
{
    if (!h || !phi) return fail(h, PIC_EINVAL, "bad argument");
    const int64_t nodes = (int64_t)(h->cfg.nr + 1) * (h->cfg.nz + 1);
    HIPCHECK(h, hipMemcpy(h->f.phi, phi, nodes * 8, hipMemcpyHostToDevice));
    if (h->prec == PIC_F64)
        launch_field_prep<double>(h->f, (double4 *)h->node, h->sc, h->cfg.scheme, 1, h->stream);
    else
        launch_field_prep<float>(h->f, (float4 *)h->node, h->sc, h->cfg.scheme, 1, h->stream);
    HIPCHECK(h, hipStreamSynchronize(h->stream));
    return PIC_OK;
}

pic_status pic_plasma_diagnostics(pic_handle *h, double r0, double r1, pic_plasma_out *out,
                                  double *maps_host)
{
    if (!h || !out) return fail(h, PIC_EINVAL, "bad argument");
    if (!(r0 < r1)) return fail(h, PIC_EINVAL, "radial band needs r0 < r1");
    return h->prec == PIC_F64 ? plasma_typed<double>(h, r0, r1, out, maps_host)
                              : plasma_typed<float>(h, r0, r1, out, maps_host);
}

pic_status pic_ied_config(pic_handle *h, double emax_ev, int32_t nbins, double r0, double r1)
{
    if (!h) return fail(nullptr, PIC_EINVAL, "handle is NULL");
    if (nbins < 0 || nbins > IED_MAX_BINS)
        return fail(h, PIC_EINVAL, "nbins outside [0, %d]", IED_MAX_BINS);
    if (nbins > 0 && (!(emax_ev > 0.0) || !(r0 < r1)))
        return fail(h, PIC_EINVAL, "the energy record needs emax_ev > 0 and r0 < r1");
    h->ied_nbins = nbins;
    h->ied_emax = emax_ev;
    h->ied_r0 = r0;
    h->ied_r1 = r1;
    launch_zero(h->pd.ied, (IED_MAX_BINS + 1) * 8, h->stream);
    HIPCHECK(h, hipStreamSynchronize(h->stream));
    return PIC_OK;
}

pic_status pic_ied_read(pic_handle *h, uint64_t *counts, int32_t ncounts, int32_t reset)
{
    if (!h || !counts) return fail(h, PIC_EINVAL, "bad argument");
    if (ncounts != h->ied_nbins + 1)
        return fail(h, PIC_EINVAL, "ncounts must be nbins + 1 = %d", h->ied_nbins + 1);
    HIPCHECK(h, hipMemcpyAsync(counts, h->pd.ied, (size_t)ncounts * 8, hipMemcpyDeviceToHost,
                               h->stream));
    if (reset) launch_zero(h->pd.ied, (IED_MAX_BINS + 1) * 8, h->stream);
    HIPCHECK(h, hipStreamSynchronize(h->stream));
    return PIC_OK;
}

pic_status pic_reweight(pic_handle *h, int32_t keep_every)
{
    if (!h) return fail(nullptr, PIC_EINVAL, "handle is NULL");
    if (keep_every < 1 || keep_every > 1000)
        return fail(h, PIC_EINVAL, "keep_every outside [1, 1000]");
    if (keep_every == 1) return PIC_OK;
    return h->prec == PIC_F64 ? reweight_typed<double>(h, keep_every)
                              : reweight_typed<float>(h, keep_every);
}

pic_status pic_compact(pic_handle *h)
{
    if (!h) return fail(nullptr, PIC_EINVAL, "handle is NULL");
    if (h->prec == PIC_F64) sort_all<double>(h);
    else sort_all<float>(h);
    return check_flags(h);
}

pic_status pic_get_state(const pic_handle *hc, pic_scalar_state *out)
{
    pic_handle *h = const_cast<pic_handle *>(hc);
    if (!h || !out) return fail(h, PIC_EINVAL, "bad argument");
    DevScalars sc;
    pic_status st = read_scalars(h, &sc);
    if (st != PIC_OK) return st;
    out->step = sc.step;
    out->vc = sc.vc;
    out->qc = sc.qc;
    out->next_id[0] = sc.next_id[0];
    out->next_id[1] = sc.next_id[1];
    out->count[0] = sc.count[0];
    out->count[1] = sc.count[1];
    out->sort_phase = h->steps_since_sort;
    out->ion_sort_phase = h->ion_sort_phase;
    return PIC_OK;
}

pic_status pic_set_state(pic_handle *h, const pic_scalar_state *in)
{
    if (!h || !in) return fail(h, PIC_EINVAL, "bad argument");
    for (int s = 0; s < 2; ++s)
        if (in->count[s] < 0 || in->count[s] > h->cap[s])
            return fail(h, PIC_EINVAL, "count out of range");
    if (in->sort_phase < 0 || in->sort_phase > h->cfg.sort_every)
        return fail(h, PIC_EINVAL, "sort_phase outside [0, sort_every]");
    if (in->ion_sort_phase < 0 || in->ion_sort_phase >= PIC_ION_SORT_EVERY)
        return fail(h, PIC_EINVAL, "ion_sort_phase outside [0, %d)", PIC_ION_SORT_EVERY);
    DevScalars sc;
    pic_status st = read_scalars(h, &sc);
    if (st != PIC_OK) return st;
    sc.step = in->step;
    sc.vc = in->vc;
    sc.qc = in->qc;
    sc.next_id[0] = in->next_id[0];
    sc.next_id[1] = in->next_id[1];
    sc.count[0] = in->count[0];
    sc.count[1] = in->count[1];
    HIPCHECK(h, hipMemcpy(h->sc, &sc, sizeof(sc), hipMemcpyHostToDevice));
    h->host_count[0] = in->count[0];
    h->host_count[1] = in->count[1];
    h->steps_since_sort = in->sort_phase;
    h->ion_sort_phase = in->ion_sort_phase;
    // phi and the gather fields from phi0 and the restored V_c
    if (h->prec == PIC_F64)
        launch_field_prep<double>(h->f, (double4 *)h->node, h->sc, h->cfg.scheme, 0, h->stream);
    else
        launch_field_prep<float>(h->f, (float4 *)h->node, h->sc, h->cfg.scheme, 0, h->stream);
    HIPCHECK(h, hipStreamSynchronize(h->stream));
    return PIC_OK;
}

pic_status pic_enable_timers(pic_handle *h, int32_t on)
{
    if (!h) return fail(nullptr, PIC_EINVAL, "handle is NULL");
    if (on < 0 || on > 2) return fail(h, PIC_EINVAL, "timer mode %d outside 0..2", (int)on);
    h->timers_on = on != 0;
    h->timers_push_only = on == 2;
    return PIC_OK;
}

pic_status pic_get_timers(pic_handle *h, pic_timers *out, int32_t reset)
{
    if (!h || !out) return fail(h, PIC_EINVAL, "bad argument");
    timers_collect(h);
    *out = h->timers;
    if (reset) h->timers = pic_timers{};
    return PIC_OK;
}

pic_status pic_apply_operator(pic_handle *h, const double *phi_dev, double *out_dev)
{
    if (!h) return fail(nullptr, PIC_EINVAL, "handle is NULL");
    if (!phi_dev || !out_dev) return fail(h, PIC_EINVAL, "phi_dev and out_dev are required");
    launch_apply_k64(h->f, phi_dev, out_dev, h->stream);
    HIPCHECK(h, hipStreamSynchronize(h->stream));
    HIPCHECK(h, hipGetLastError());
    return PIC_OK;
}

pic_status pic_pc_param_count(int64_t *n)
{
    if (!n) return fail(nullptr, PIC_EINVAL, "n is NULL");
    PcNet t;
    pc_describe(t, 4, 4, 1);
    *n = t.n_flat;
    return PIC_OK;
}

pic_status pic_pc_set_weights(pic_handle *h, const float *theta, int64_t n, double out_scale)
{
    if (!h) return fail(nullptr, PIC_EINVAL, "handle is NULL");
    if (!h->pc_on) return fail(h, PIC_ESTATE, "no learned-preconditioner buffers (pc_batch = 0)");
    if (!theta || n != h->net.n_flat)
        return fail(h, PIC_EINVAL, "expected %lld parameters", (long long)h->net.n_flat);
    if (!std::isfinite(out_scale) || !(out_scale > 0.0))
        return fail(h, PIC_EINVAL, "out_scale must be positive and finite");
    for (int64_t k = 0; k < n; ++k)
        if (!std::isfinite(theta[k])) return fail(h, PIC_EINVAL, "parameter %lld is not finite", (long long)k);
    HIPCHECK(h, hipStreamSynchronize(h->stream));
    // cached solve graphs hold the output scale by value
    drop_graphs(h);
    h->net.out_scale = out_scale;
    pc_upload(h->net, theta, h->stream);
    HIPCHECK(h, hipStreamSynchronize(h->stream));
    HIPCHECK(h, hipGetLastError());
    h->net.has_weights = true;
    return PIC_OK;
}

pic_status pic_pc_get_weights(pic_handle *h, float *theta, int64_t n, double *out_scale)
{
    if (!h) return fail(nullptr, PIC_EINVAL, "handle is NULL");
    if (!h->pc_on || !h->net.has_weights) return fail(h, PIC_ESTATE, "no weights loaded");
    if (!theta || n != h->net.n_flat)
        return fail(h, PIC_EINVAL, "expected %lld parameters", (long long)h->net.n_flat);
    HIPCHECK(h, hipStreamSynchronize(h->stream));
    std::vector<float> tmp;
    pc_download_flat(h->net, h->net.master, theta, tmp);
    if (out_scale) *out_scale = h->net.out_scale;
    return PIC_OK;
}

pic_status pic_pc_train_step(pic_handle *h, const double *q_dev, const double *phi_dev,
                             int32_t batch, float lr, double *loss, float *grad)
{
    if (!h) return fail(nullptr, PIC_EINVAL, "handle is NULL");
    if (!h->pc_on || !h->net.has_weights) return fail(h, PIC_ESTATE, "no weights loaded");
    if (!q_dev || !phi_dev) return fail(h, PIC_EINVAL, "q_dev and phi_dev are required");
    if (batch < 1 || batch > h->net.batch)
        return fail(h, PIC_EINVAL, "batch %d outside [1, %d]", batch, h->net.batch);
    if (!(lr >= 0.0f) || !std::isfinite(lr)) return fail(h, PIC_EINVAL, "lr must be >= 0");
    const double inv_2pi_eps0 = 1.0 / (2.0 * 3.14159265358979323846 * eps0());
    pc_train_enqueue(h->net, pc_pre_of(h), h->f.mg.lv[0], h->n_unknown, q_dev, phi_dev, batch, lr, inv_2pi_eps0,
                     h->stream);
    double l = 0.0;
    HIPCHECK(h, hipMemcpyAsync(&l, pc_loss_ptr(h->net, batch), 8, hipMemcpyDeviceToHost,
                               h->stream));
    HIPCHECK(h, hipStreamSynchronize(h->stream));
    HIPCHECK(h, hipGetLastError());
    if (loss) *loss = l;
    if (grad) {
        std::vector<float> tmp;
        pc_download_flat(h->net, h->net.grad, grad, tmp);
    }
    if (!std::isfinite(l)) return fail(h, PIC_ENAN, "non-finite training loss");
    return PIC_OK;
}

pic_status pic_pc_apply(pic_handle *h, const double *r_dev, double *z_dev)
{
    if (!h) return fail(nullptr, PIC_EINVAL, "handle is NULL");
    if (!h->pc_on || !h->net.has_weights) return fail(h, PIC_ESTATE, "no weights loaded");
    if (!r_dev || !z_dev) return fail(h, PIC_EINVAL, "r_dev and z_dev are required");
    pc_apply64(h->net, pc_pre_of(h), h->f.mg.lv[0], h->n_unknown, r_dev, z_dev, &h->sc->pcg_ss[MAX_PCG + 1],
               h->stream);
    HIPCHECK(h, hipStreamSynchronize(h->stream));
    HIPCHECK(h, hipGetLastError());
    return PIC_OK;
}

pic_status pic_set_poisson_mode(pic_handle *h, int32_t mode)
{
    if (!h) return fail(nullptr, PIC_EINVAL, "handle is NULL");
    if (mode != PIC_MGCG && mode != PIC_LEARNED && mode != PIC_CG && mode != PIC_DIRECT)
        return fail(h, PIC_EINVAL, "mode must be PIC_MGCG, PIC_LEARNED, PIC_CG or PIC_DIRECT");
    if (mode == PIC_LEARNED && !h->pc_on)
        return fail(h, PIC_ESTATE, "no learned-preconditioner buffers (pc_batch = 0)");
    if (mode == PIC_DIRECT && !h->fs_on)
        return fail(h, PIC_ESTATE, "no direct-solve buffers (created with another poisson_mode)");
    h->pmode = mode;
    return PIC_OK;
}

pic_status pic_ensemble_create(pic_handle *const *runs, int32_t nruns, void *stream,
                               int32_t nstreams, pic_ensemble **out)
{
    if (!out) return efail(nullptr, PIC_EINVAL, "out is NULL");
    *out = nullptr;
    if (!runs || nruns < 1) return efail(nullptr, PIC_EINVAL, "no runs");
    if (nstreams < 1 || nstreams > 16) return efail(nullptr, PIC_EINVAL, "nstreams outside [1, 16]");
    for (int r = 0; r < nruns; ++r) {
        const pic_handle *h = runs[r];
        if (!h) return efail(nullptr, PIC_EINVAL, "run %d is NULL", r);
        for (int q = 0; q < r; ++q)
            if (runs[q] == h) return efail(nullptr, PIC_EINVAL, "run %d appears twice", r);
        if (h->cfg.sort_every != runs[0]->cfg.sort_every)
            return efail(nullptr, PIC_EINVAL, "run %d: every run must share sort_every", r);
        if (h->prec != runs[0]->prec)
            return efail(nullptr, PIC_EINVAL, "run %d: every run must share the state precision", r);
        if (!h->cfg.field_solve)
            return efail(nullptr, PIC_EINVAL, "run %d: ensembles solve the field every step", r);
        if (h->cfg.deposit_fixed)
            return efail(nullptr, PIC_EINVAL, "run %d: the fixed-point deposit is a single-run mode",
                         r);
        if (h->timers_on) return efail(nullptr, PIC_EINVAL, "run %d: timers must be off", r);
    }
    pic_ensemble *e = new pic_ensemble();
    e->plans.clear();
    e->runs.assign(runs, runs + nruns);
    if (stream) {
        e->s0 = (hipStream_t)stream;
    } else {
        if (hipStreamCreateWithFlags(&e->s0, hipStreamNonBlocking) != hipSuccess) {
            delete e;
            return efail(nullptr, PIC_EHIP, "cannot create a stream");
        }
        e->own_s0 = true;
    }
    bool ok = true;
    const int nbatch = (nruns + MAX_BATCH - 1) / MAX_BATCH;
    ok &= hipHostMalloc((void **)&e->status, sizeof(RunStatus) * nbatch * MAX_BATCH) == hipSuccess;
    ok = ok && hipHostGetDevicePointer((void **)&e->status_dev, e->status, 0) == hipSuccess;
    if (!ok) {
        pic_ensemble_free(e);
        return efail(nullptr, PIC_EHIP, "cannot create the ensemble's status buffer");
    }
    memset(e->status, 0, sizeof(RunStatus) * nbatch * MAX_BATCH);
    // the descriptor of each run's batched field update, in its workspace
    e->plans.resize(nbatch);
    const double inv_2pi_eps0 = 1.0 / (2.0 * 3.14159265358979323846 * eps0());
    for (int r = 0; r < nruns; ++r) {
        pic_handle *h = e->runs[r];
        const pic_config &c = h->cfg;
        RunSolve R;
        memset(&R, 0, sizeof(R));
        R.f = h->f;
        const int32_t *g = &h->sc->solve_done;
        R.f.gate = g;
        for (int l = 0; l < MAX_LEVELS; ++l) {
            R.f.mg.lv[l].gate = g;
            R.f.mg.tail.L[l].gate = g;
        }
        R.sc = h->sc;
        R.q0 = h->q[0];
        R.q1 = h->q[1];
        R.node = h->node;
        R.rtol2 = c.poisson_rtol * c.poisson_rtol;
        R.v_fixed = c.v_fixed;
        R.v_ext = c.v_ext;
        R.r_ext = c.r_ext;
        R.dt = c.dt;
        R.extra_dq = c.extra_current * c.dt;
        R.inv_2pi_eps0 = inv_2pi_eps0;
        R.circuit = c.circuit;
        R.scheme = c.scheme;
        R.cg.r[0] = h->f.mg.lv[0].b;
        R.cg.r[1] = h->f.r32b;
        R.cg.q[0] = h->f.q32;
        R.cg.q[1] = h->f.q32b;
        R.cg.w = h->f.w32;
        R.cg.p = h->f.p32[0];
        R.cg.e = h->f.e32;
        R.cg.acc = h->f.cg_acc;
        R.cg.pq = h->sc->pcg_pq;
        if ((const char *)h->rsolve + sizeof(RunSolve) > h->ws + h->ws_bytes) {
            pic_ensemble_free(e);
            return efail(nullptr, PIC_EINVAL, "run %d: no room for the run descriptor", r);
        }
        if (hipMemcpy(h->rsolve, &R, sizeof(R), hipMemcpyHostToDevice) != hipSuccess) {
            pic_ensemble_free(e);
            return efail(nullptr, PIC_EHIP, "cannot upload the run descriptors");
        }
        // particle-kernel parameters for each pair of current buffers
        if (h->part_desc + 4 * PART_DESC_BYTES > h->ws + h->ws_bytes) {
            pic_ensemble_free(e);
            return efail(nullptr, PIC_EINVAL, "run %d: no room for the particle descriptors", r);
        }
        const bool up = h->prec == PIC_F64 ? upload_run_particles<double>(h)
                                           : upload_run_particles<float>(h);
        if (!up) {
            pic_ensemble_free(e);
            return efail(nullptr, PIC_EHIP, "cannot upload the particle descriptors");
        }
        BatchPlan &P = e->plans[r / MAX_BATCH];
        P.dev[P.nruns] = h->rsolve;
        P.host[P.nruns] = h->f.mg;
        P.nruns++;
        P.prec = h->prec;
    }
    // one sort phase for all: cell-sort every run now, twice where that
    // leaves its particles in the other buffer of the pair than run 0's
    for (int r = 0; r < nruns; ++r) {
        pic_handle *h = e->runs[r];
        for (int k = 0; k < 2; ++k) {
            if (k == 1 && h->cur[0] == e->runs[0]->cur[0] && h->cur[1] == e->runs[0]->cur[1]) break;
            if (h->prec == PIC_F64) sort_all<double>(h);
            else sort_all<float>(h);
        }
        const hipError_t es = hipStreamSynchronize(h->stream);
        if (es != hipSuccess) {
            pic_ensemble_free(e);
            return efail(nullptr, PIC_EHIP, "run %d: sort before the first step failed: %s", r,
                         hipGetErrorString(es));
        }
    }
    *out = e;
    return PIC_OK;
}

pic_status pic_ensemble_step(pic_ensemble *e, int32_t nsteps)
{
    if (!e) return efail(nullptr, PIC_EINVAL, "ensemble is NULL");
    if (nsteps < 0) return efail(e, PIC_EINVAL, "nsteps < 0");
    for (int k = 0; k < nsteps; ++k) {
        pic_status st = ensemble_step(e);
        if (st != PIC_OK) return st;
    }
    return PIC_OK;
}

pic_status pic_ensemble_free(pic_ensemble *e)
{
    if (!e) return PIC_OK;
    if (e->s0) (void)hipStreamSynchronize(e->s0);
    drop_ensemble_graphs(e);
    if (e->status) (void)hipHostFree(e->status);
    if (e->own_s0 && e->s0) (void)hipStreamDestroy(e->s0);
    delete e;
    return PIC_OK;
}

const char *pic_ensemble_last_error(const pic_ensemble *e)
{
    if (!e) return g_init_error.c_str();
    return e->err.c_str();
}

pic_status pic_set_tuning(pic_handle *h, const pic_tuning *t)
{
    if (!h || !t) return fail(h, PIC_EINVAL, "NULL argument");
    if (t->push_blocks < 2 || t->push_blocks > 65536 || !(t->push_e_weight > 0.0) ||
        !(t->push_e_weight < 100.0))
        return fail(h, PIC_EINVAL, "push_blocks in [2, 65536] and push_e_weight in (0, 100)");
    if (t->mg_one_level != 0 && t->mg_one_level != 1)
        return fail(h, PIC_EINVAL, "mg_one_level must be 0 or 1");
    if (t->pass_graphs != 0 && t->pass_graphs != 1)
        return fail(h, PIC_EINVAL, "pass_graphs must be 0 or 1");
    h->push_blocks = t->push_blocks;
    h->push_e_weight = t->push_e_weight;
    if (h->mg_one_level != (t->mg_one_level != 0)) {
        h->mg_one_level = t->mg_one_level != 0;
        drop_graphs(h);   // captured solves hold the other launch sequence
    }
    if (h->use_graphs != (t->pass_graphs != 0)) {
        h->use_graphs = t->pass_graphs != 0;
        drop_graphs(h);
    }
    return PIC_OK;
}

pic_status pic_get_tuning(const pic_handle *h, pic_tuning *t)
{
    if (!h || !t) return fail(nullptr, PIC_EINVAL, "NULL argument");
    memset(t, 0, sizeof(*t));
    t->push_blocks = h->push_blocks;
    t->push_e_weight = h->push_e_weight;
    t->mg_one_level = h->mg_one_level ? 1 : 0;
    t->pass_graphs = h->use_graphs ? 1 : 0;
    return PIC_OK;
}

pic_status pic_autotune(pic_handle *h, int32_t steps_per_trial, void *scratch_dev,
                        int64_t scratch_bytes, pic_tuning *out)
{
    if (!h) return fail(nullptr, PIC_EINVAL, "handle is NULL");
    if (steps_per_trial < 1) return fail(h, PIC_EINVAL, "steps_per_trial < 1");
    const int64_t snap_bytes = layout(h->cfg, nullptr, nullptr);
    if (scratch_dev && scratch_bytes < snap_bytes)
        return fail(h, PIC_EINVAL, "autotune scratch of %lld bytes < %lld needed",
                    (long long)scratch_bytes, (long long)snap_bytes);
    const bool was_on = h->timers_on, was_push_only = h->timers_push_only;
    HIPCHECK(h, hipStreamSynchronize(h->stream));
    timers_collect(h);
    const pic_timers saved = h->timers;
    // The trials step the live simulation.  With scratch, its state is
    // copied first (the workspace into the caller's buffer, the handle's
    // host-side solver state) and put back afterwards, so tuning leaves the
    // run where it was.
    char *snap = (char *)scratch_dev;
    if (snap)
        HIPCHECK(h, hipMemcpyAsync(snap, h->ws, (size_t)snap_bytes, hipMemcpyDeviceToDevice,
                                   h->stream));
    const int cur0[2] = {h->cur[0], h->cur[1]};
    const int64_t count0[2] = {h->host_count[0], h->host_count[1]};
    const int sort0 = h->steps_since_sort, ion_sort0 = h->ion_sort_phase;
    const pic_poisson_stats last0 = h->last;
    const double rho0 = h->rho, rel00 = h->rel0_est, rho_pc0 = h->rho_pc, rho_cg0 = h->rho_cg;
    const int32_t flags0 = h->host_flags;
    h->timers_on = true;
    h->timers_push_only = true;
    // one trial: the mean device time of the particle kernel over the steps
    auto trial = [&](int blocks, double w, double *ms) -> pic_status {
        h->push_blocks = blocks;
        h->push_e_weight = w;
        h->timers = pic_timers{};
        pic_status st = pic_step(h, steps_per_trial);
        if (st != PIC_OK) return st;
        HIPCHECK(h, hipStreamSynchronize(h->stream));
        timers_collect(h);
        *ms = h->timers.push_ms / std::max<int64_t>(h->timers.push_launches, 1);
        return PIC_OK;
    };
    pic_tuning best = {h->push_blocks, h->push_e_weight, 1e300, 0, h->mg_one_level ? 1 : 0,
                       h->use_graphs ? 1 : 0};
    pic_status st = PIC_OK;
    // coordinate search: block count at the current weight, then the weight
    static const int blocks[] = {256, 512, 1024, 2048, 4096, 8192};
    static const double weights[] = {1.0, 1.3, 1.7};
    for (int b : blocks) {
        double ms;
        if ((st = trial(b, best.push_e_weight, &ms)) != PIC_OK) break;
        if (ms < best.push_ms) {
            best.push_ms = ms;
            best.push_blocks = b;
        }
    }
    if (st == PIC_OK)
        for (double w : weights) {
            double ms;
            if ((st = trial(best.push_blocks, w, &ms)) != PIC_OK) break;
            if (ms < best.push_ms) {
                best.push_ms = ms;
                best.push_e_weight = w;
            }
        }
    h->push_blocks = best.push_blocks;
    h->push_e_weight = best.push_e_weight;
    // back to the saved state
    hipError_t e = hipStreamSynchronize(h->stream);
    if (snap) {
        if (e == hipSuccess)
            e = hipMemcpyAsync(h->ws, snap, (size_t)snap_bytes, hipMemcpyDeviceToDevice, h->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
        h->cur[0] = cur0[0];
        h->cur[1] = cur0[1];
        h->host_count[0] = count0[0];
        h->host_count[1] = count0[1];
        h->steps_since_sort = sort0;
        h->ion_sort_phase = ion_sort0;
        h->last = last0;
        h->rho = rho0;
        h->rel0_est = rel00;
        h->rho_pc = rho_pc0;
        h->rho_cg = rho_cg0;
        h->host_flags = flags0;
    }
    timers_collect(h);
    h->timers = saved;
    h->timers_on = was_on;
    h->timers_push_only = was_push_only;
    if (e != hipSuccess) return fail(h, PIC_EHIP, "autotune: %s", hipGetErrorString(e));
    if (st != PIC_OK) return st;
    best.trials = (int32_t)(sizeof(blocks) / sizeof(blocks[0]) + sizeof(weights) / sizeof(weights[0]));
    if (out) *out = best;
    return PIC_OK;
}

pic_status pic_free(pic_handle *h)
{
    if (!h) return PIC_OK;
    (void)hipStreamSynchronize(h->stream);
    timers_collect(h);
    for (auto &g : h->graphs) (void)hipGraphExecDestroy(g.exec);
    for (auto &e : h->free_events) {
        (void)hipEventDestroy(e.first);
        (void)hipEventDestroy(e.second);
    }
    if (h->pinned) (void)hipHostFree(h->pinned);
    if (h->rb_done) (void)hipEventDestroy(h->rb_done);
    delete h;
    return PIC_OK;
}

const char *pic_last_error(const pic_handle *h)
{
    if (!h) return g_init_error.c_str();
    return h->err.c_str();
}

}  // extern "C"
