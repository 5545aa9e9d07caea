// Learned preconditioner of the field solve: a 4-level U-Net f (15 3x3
// convolutions, 196,753 parameters) whose correction out_scale rms(r1)
// f(r1 / rms(r1), i / 256) of a pre-smoothed residual r1 sits between
// red-black Gauss-Seidel sweeps, inside flexible conjugate gradients; and its
// training (relative A-norm error loss, backward pass, Adam) on pairs
// (Q, phi) with K phi = Q, pre-smoothed the same way.
//
// Activations are FP32, NHWC: [batch][H][W][C_p], C_p = channels rounded up
// to 4, the padding channels always zero; level l has H_l x W_l nodes with
// H_0 = nz + 1, W_0 = nr + 1 and H_{l+1} = ceil(H_l / 2).  Convolutions run
// on BF16 MFMA with FP32 accumulation.
//
// Weights: one FP32 "master" matrix per layer, rows = output channels padded
// to a multiple of 16, row length kw = roundup(9 cin_p + 1, 16), column
// k = tap * cin_p + c (tap = 3 kh + kw) for the weight w[n][c][kh][kw] and
// column 9 cin_p for the bias.  From it the BF16 copies used by the kernels:
// forward rows [n][kpad] and data-gradient rows [c][kpad_t] of the flipped
// kernel, k' = tap' * cout_p + n holding w[n][c][8 - tap'].
#pragma once

#include "common.h"

namespace pic {

constexpr int PC_LAYERS = 15;
constexpr int PC_LEVELS = 4;
constexpr int PC_WGRAD_SPLITS = 2048;  // most pixel ranges of the weight-gradient kernel

struct PcLayer {
    int32_t cin, cout;          // channels
    int32_t cin_p, cout_p;      // padded to 4
    int32_t level;              // level of the output
    int32_t up_in;              // input is the coarser level, read nearest-neighbour
    int32_t relu;
    int32_t kpad;               // forward BF16 row length (9 cin_p rounded up to 32)
    int32_t kpad_t;             // data-gradient BF16 row length (9 cout_p rounded up to 32)
    int32_t kw;                 // master row length (bias at column 9 cin_p)
    int32_t nt, nt_t;           // 16-row tiles of cout, of cin
    int64_t o_master;           // offsets: master / gradient / Adam (floats)
    int64_t o_wf, o_wt;         // BF16 copies (shorts)
    int64_t o_bias;             // FP32 bias copy (floats)
    int64_t o_flat;             // flat [cout][cin][3][3] + [cout] parameter vector
};

struct PcNet {
    PcLayer L[PC_LAYERS];
    int32_t H[PC_LEVELS], W[PC_LEVELS];
    int32_t batch;
    int64_t n_master, n_flat;
    float *master, *grad, *adam_m, *adam_v, *bias;
    short *wf, *wt;
    float *partial;
    // activations
    float *x, *c0a, *e0, *d0a, *d0, *out;
    float *p1, *c1a, *e1, *d1a, *d1;
    float *p2, *c2a, *e2, *d2a, *d2;
    float *p3, *c3a, *e3;
    // gradients (see pc_backward for the reuse of each buffer)
    float *g_out, *gA0, *gS0;
    float *gA1, *gS1, *gB1, *gP1;
    float *gA2, *gS2, *gB2, *gP2;
    float *gA3, *gC3, *gP3;
    float *tgt;                 // [batch][P0] scaled targets
    float *vb, *vx, *vr, *vz;   // [batch][P0] FP32 node vectors: right-hand side,
                                // pre-smoothed iterate, its residual, output
    double *scal;               // [4][batch] sums (see pc_train_enqueue)
    int32_t adam_t;
    double out_scale;
    bool has_weights;
};

// Layer table and workspace.  pc_bytes is the size pc_bind carves from base.
void pc_describe(PcNet &n, int nr, int nz, int batch);
int64_t pc_bytes(const PcNet &n);
void pc_bind(PcNet &n, char *base);
int pc_kernel_setup();          // raises the dynamic-LDS limit of the conv kernels
bool pc_fits(const PcNet &n);  // every convolution's block fits a CU's LDS

// Flat parameters (host) <-> master (device); builds the BF16 copies, zeroes Adam.
void pc_upload(PcNet &n, const float *flat, hipStream_t s);
void pc_download_flat(const PcNet &n, const float *dev_master_like, float *flat_host,
                      std::vector<float> &tmp);
void pc_pack(const PcNet &n, hipStream_t s);

// Where the preconditioner's first approximation x1 of A x = r comes from:
// a red-black Gauss-Seidel pair from zero (red, black), or one multigrid
// V-cycle of the hierarchy H (the multigrid preconditioner of the solver;
// it reads H.lv[0].b and writes H.lv[0].xu).
struct PcPre {
    const MGHier *H;            // nullptr: the Gauss-Seidel pair
    bool two_level;
};

// Preconditioner application inside the FP32 CG on level L (the finest
// multigrid level): x1 from `pre`, r1 = r - A x1, z = x1 + out_scale rho1
// f(r1 / rho1) with rho1 the rms of r1 over the unknowns, then a black and a
// red sweep on A z = r.  Accumulates r.z into *rz and, when q is given, z.q
// into *zq; *ss must be zero on entry (rms accumulator).  Enqueue only.
void pc_apply32(PcNet &n, const PcPre &pre, const MGLevel &L, int64_t n_unknown, const float *r,
                float *z, const float *q, double *rz, double *zq, double *ss, hipStream_t s);
void pc_apply64(PcNet &n, const PcPre &pre, const MGLevel &L, int64_t n_unknown, const double *r,
                double *z, double *ss, hipStream_t s);
// identity "preconditioner" of plain CG: z = r, *rz += r.r
void pc_identity32(const MGLevel &L, const float *r, float *z, double *rz, hipStream_t s);

// One training step on B pairs (q node charges in C, phi in V, FP64,
// [B][nodes], zero on Dirichlet nodes): b = q / (2 pi eps0) scaled to unit
// rms, x1 = pre-smoothing of b, network input r1 = b - A x1 (unit rms), target
// (phi / rms(b) - x1) / rms(r1); forward, loss, backward, Adam.  Leaves the
// gradient in n.grad and the batch loss at pc_loss_ptr.
void pc_train_enqueue(PcNet &n, const PcPre &pre, const MGLevel &L, int64_t n_unknown,
                      const double *q, const double *phi, int B, float lr, double inv_2pi_eps0,
                      hipStream_t s);
const double *pc_loss_ptr(const PcNet &n, int B);

}  // namespace pic
