// Host-side interfaces between the ABI layer and the kernels of libcvbound.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"

namespace cvb {

// Per-kernel timing (the eager timing pass only; never during graph capture):
// when `start` is set, the next kernel launch on this host thread is issued
// `reps` times back to back between `start` and `stop` recorded on its stream,
// then the request is cleared.  Repeats take the same arguments, so they touch
// exactly the memory of the first launch.
struct LaunchTiming {
  hipEvent_t start = nullptr, stop = nullptr;
  int reps = 1;
};
LaunchTiming& launch_timing();

template <typename... P, typename... A>
inline void launch_k(void (*k)(P...), dim3 grid, dim3 block, uint32_t smem, hipStream_t s, A... args) {
  LaunchTiming& t = launch_timing();
  if (t.start) {
    const LaunchTiming req = t;
    t = LaunchTiming{};
    (void)hipEventRecord(req.start, s);
    for (int r = 0; r < req.reps; ++r) k<<<grid, block, smem, s>>>(args...);
    (void)hipEventRecord(req.stop, s);
  } else {
    k<<<grid, block, smem, s>>>(args...);
  }
}

// Epilogue / prologue variants of the layer kernels.
enum Mode {
  kBwdRelax = 0,  // back-substitution, then the next ReLU layer's relaxation
  kBwdConc = 1,   // back-substitution into the input, then box concretisation
  kFwdX = 2,      // adjoint forward step from x* of a conv first layer (its sign planes)
  kFwd = 3,       // adjoint forward step from zhat(i-1)
  kFwdTop = 4     // kFwd for the top ReLU layer inside the optimiser, plus the
                  // next iteration's top-layer relaxation (Epi::top_out)
};

struct GemmCfg {
  int bm, bn, bk;
  int occ;    // minimum waves per SIMD requested from the compiler (0: its choice)
  int depth;  // K slabs of global loads in flight (1, 2, or all of K when >= 3)
};
constexpr int kNumGemmCfgs = 40;
extern const GemmCfg kGemmCfgs[kNumGemmCfgs];
// whether tiling `cfg` can run a contraction of depth K (all-of-K tilings
// hold K <= depth * bk); launch_gemm substitutes a two-deep tiling otherwise
bool gemm_cfg_fits(int cfg, int K);

struct GemmArgs {
  const float* A;
  int lda;
  const float* Bt;
  int ldb;
  int M, N, K;
  int last;  // adjoint: do not write zhat (the top ReLU layer)
  Batch bt;
  Vars v;
  Epi e;
};
void launch_gemm(int cfg, int mode, const GemmArgs& g, hipStream_t s);

struct ConvGeom {
  int ci, hi, wi, co, ho, wo, k, s, p;
};
// One direction of a conv layer as an implicit GEMM per batch row,
// D[m, n] = sum_k G[m, k] Wm[k, n] (conv.hip).  The row's input is staged
// in LDS with a zero border around each gh x gw channel plane (padded row
// width gwp, padded plane pplane, interior origin bofs), so that G[m, k] is
// staged[m.x + k.x] with no range check.  D[m, n] is
// output[n.z + (osy * m.z + n.x) * ow + (osx * m.w + n.y)] when that lies in
// the oh x ow plane and n.z >= 0.  Device tables, built once per layer.
struct ConvPlan {
  const int4* mtab;  // [mpad] gather offset x and output origin (z, w) of GEMM row m
  const int4* ktab;  // [kpad] gather offset x of GEMM column k
  const int4* ntab;  // [16 nt] output offset (x, y) and channel base z (-1: padding)
  // [kpad / 4] or null: when the column offsets split as ktab[4 s + q].x =
  // kuni[s] + v(q) (a per-step part uniform across the wave and a per-lane
  // part; in-range taps for the padding columns), the GEMM gathers through
  // kuni, read by scalar loads, and v, instead of reading ktab every step
  const int* kuni;
  const float* wm;   // [kpad / 4][nt][64] Wm in MFMA 16x16x4 operand order
  int mpad, kpad, nt;  // multiples of 16; nt: 16-column tiles (1, 2, 4 or 8)
  int gh, gw;          // gathered plane
  int oh, ow, osy, osx;  // output plane and its stride factors
  int din, dout;       // input and output floats per row
  int dinp;            // staged floats per row (with the zero borders)
  int gwp, pplane, bofs;  // padded row width, padded plane, offset of the interior origin
  unsigned mgp, mgw;   // ceil(2^32 / (gh gw)), ceil(2^32 / gw): exact division of staging indices
  int wg;              // 1: the kernel reads wm from global memory, not LDS
  int grid;            // persistent workgroups
  int smem;            // dynamic LDS bytes
  // subdomain-major kernel (conv_sd): outputs and inputs per thread held in
  // registers (0: no instantiation holds this layer), its persistent
  // workgroups, and whether launches use it (else the row-major conv_mm)
  int nj, ni;
  int grid_sd;
  int smem_sd;  // its dynamic LDS bytes (the plan's and the layer's bias per neuron)
  int sd;
};
struct ConvArgs {
  const float* in;
  int ldi;
  ConvPlan pl;
  int M;
  int last;
  Batch bt;
  Vars v;
  Epi e;
};
// LDS bytes of a plan and the workgroups that run concurrently on the device
int conv_plan_smem(const ConvPlan& pl);
int conv_plan_grid(int mode, const ConvPlan& pl);
// register sizes of the subdomain-major kernel for a plan (nj = ni = 0 when
// no instantiation holds it) and its concurrent workgroups
void conv_plan_sd(int mode, ConvPlan& pl);
// Kernel variant of a conv plan: 0 row-major with the weights in LDS, 1
// row-major reading them from global memory, 2 and 3 the subdomain-major
// kernel likewise.  Rebuilds the LDS size and grids; -1 (plan unchanged)
// when the variant cannot run this layer.
constexpr int kNumConvVariants = 4;
int conv_plan_variant(int mode, ConvPlan& pl, int variant);
int launch_convt_bwd(int mode, const ConvArgs& a, hipStream_t s);
int launch_conv_fwd(int mode, const ConvArgs& a, hipStream_t s);

// chain.hip: runs of dense layers fused per row tile
struct ChainLayer {
  const float* Bt;     // K-contiguous operand [N, ldb] (back-substitution: W^T; adjoint: W)
  int ldb;
  int K, N;
  const float* bias;   // bias of the output layer (per neuron)
  int out_off;         // nd offset of the output ReLU layer (unused when concretising)
};
constexpr int kChainMax = 12;
struct ChainArgs {
  int nl;
  ChainLayer ly[kChainMax];
  int np;    // LDS pitch basis: widest LDS-resident operand rounded to 32
  int ncw;   // output columns per chunk: that width rounded to 16
  int ldk;   // LDS row stride of the resident rows (np + 4 floats)
  int rb;    // 16-row MFMA blocks per workgroup (1..kChainRowBlocks)
  int uw;    // 16x16 output units per wave: ceil(rb * ncw/16 / 8)
  int grid;  // workgroups; rows divided evenly over them
  // back-substitution start: the top ReLU layer from C W(L)
  const float* CW;
  int64_t cw_pstride;
  int ldcw;
  const float* Cb;
  int64_t cb_pstride;
  int n_top;
  int top_off;
  const float* top_bias;
  int conc;  // 1: the last step concretises into the input; 0: write relaxed Lambda to out
  // adjoint start: 1 = x* from the sign planes, 0 = read `in`
  int from_x;
  const float* in;
  int ldi;
  float* out;
  int ldo;
  float* part;
  int n_slots;
  int slot;
  float* lb;
  float* best;
  int first;
  int final;  // 1: the chain completes the pass: write lb / best instead of a slot
  Batch bt;
  Vars v;
};
constexpr int kChainRowBlocks = 3;  // 16-row MFMA blocks per chain workgroup, at most
size_t chain_smem_bytes(int rb, int np);
bool chain_units_fit(int rb, int np, int ncw);
int chain_units_per_wave(int rb, int ncw);
void chain_prepare(int lds_bytes);
void launch_chain_bwd(const ChainArgs& a, hipStream_t s);
void launch_chain_fwd(const ChainArgs& a, hipStream_t s);

// sound64.hip: the sound-mode evaluation in float64
struct Pass64 {
  Batch bt;
  const float* l;      // [P, nd] root bounds (the chords are formed from them in double)
  const float* u;
  const float* alpha;  // [n_alpha] or null (default slopes)
  const float* beta;   // [nnz, m]
  const float* sw;     // [P, nd] weight of |Lambda_k| in the float64 rounding-error bound
  double sg;           // weight of each concretisation term
  double* part;        // [slots, R] partial constants
  double* perr;        // [slots, R] partial rounding-error bounds
  double* psq;         // [slots, R] partial sums of A(0)^2 (l2 ball), or null
};
struct Top64 {
  // general specification: C_p [m, dL] times the last (dense) layer W(L),
  // b(L), formed in double; or (C null) the exact float rows CW = +-W(L)
  const float* C;
  int dL;
  const float* WL;
  int ldw;
  const float* bL;
  const float* CW;
  int64_t cw_pstride;
  int ldcw;
  const float* Cb;
  int64_t cb_pstride;
  int n;            // width of layer L-1
  int layer_off;
  const float* bias;  // bias of layer L-1 per neuron
  double* out;
  int ldo;
  int conc;         // no ReLU layer: concretise directly
  const float* err0;  // [P, m] rounding-error bound of forming C W(L) and C b(L)
};
struct Lay64 {
  const double* in;  // Lambda(i) rows
  int ldi;
  int K, N;          // d_i, d_(i-1)
  const float* W;    // dense [d_i, ldw]; conv OIHW
  int ldw;
  int conc;          // 1: into the input (concretise)
  int layer_off;     // layer i-1 in the nd axis (relaxation)
  const float* bias; // bias of layer i-1 per neuron
  double* out;
  int ldo;
  int slot;
};
struct Fin64 {
  int n_used;
  double scale;      // >= 1: the summation of the error partials
  double ball;       // relative rounding of ||A(0)||_2 and of the A(0) x0 sum (l2 ball)
  const float* x0n;  // [P] ||x0||_2 rounded up (l2 ball)
  float* lb;
  float* best;
  int first;
};
void launch_top64(const Pass64& q, const Top64& t, hipStream_t s);
void launch_dense64(const Pass64& q, const Lay64& y, hipStream_t s);
void launch_conv64(const Pass64& q, const Lay64& y, const ConvGeom& g, hipStream_t s);
void launch_finalize64(const Pass64& q, const Fin64& f, hipStream_t s);

// misc.hip
void launch_prep_chord(const float* l, const float* u, float2* chord, float* adef, int64_t n, hipStream_t s);
void launch_status_fill(uint32_t* status, const uint32_t* root_kind, const int* prop, int B, int nd,
                        hipStream_t s);
void launch_status_split(uint32_t* status, const int* split_dom, const int* split_col, const int8_t* side,
                         int64_t nnz, int nd, hipStream_t s);
void launch_spec_merge(const float* C, const float* W, int ldw, const float* b, int P, int m, int dL, int dprev,
                       float* CW, int ldcw, float* Cb, hipStream_t s);
void launch_spec_identity(const float* Wdense, int ldw, const float* wconv, const ConvGeom* g,
                          const float* bias_full, int d, int dprev, float* CW, int ldcw, float* Cb, hipStream_t s);
struct TopArgs {
  const float* CW;
  int64_t cw_pstride;  // floats between properties (0: shared by all)
  int ldcw;
  const float* Cb;
  int64_t cb_pstride;
  int n;       // width of layer L-1
  int conc;    // 1 when there is no ReLU layer: concretise directly
  const float* err0;  // sound mode: rounding-error constant of the merged specification [P, m], or null
  Batch bt;
  Vars v;
  Epi e;
};
void launch_top(const TopArgs& a, hipStream_t s);
// ub[row] = C_p W(L) z[row] + C_p b(L), z = zhat(L-1) of the network at x*
void launch_top_dot(const TopArgs& a, const float* z, int ldz, float* ub, hipStream_t s);
void launch_fill_i32(int* p, int v, int64_t n, hipStream_t s);
// l_p-ball concretisation data of the final sum
struct L2Final {
  const int* prop;    // [B] property of each subdomain
  int m;              // rows per subdomain
  const float* eps;   // [P] radius
  float* l2s;         // [n_rows] out: eps / ||A(0)||_q^(q-1), or null
  // sound mode: ||x0_p||_2 rounded up [P], the concretisation sum's error
  // factor g, and fac >= 1 bounding the rounding of the norm (unused otherwise)
  const float* x0n;
  float g, fac;
  float q;  // dual exponent of the ball (2: l2; sound mode only with 2)
};
// lb = sum of the used partial slots of each row; with perr (sound mode) minus
// `scale` times the sum of the rounding-error partials, rounded outward; with
// psq (l_p ball) minus eps_p (sum of the |A(0)|^q partials)^(1/q)
// improved (optional, with best): improved[row] = 1 where this bound raised
// best[row] (or first), else 0
void launch_finalize(const float* part, const float* perr, float scale, const float* psq, const L2Final& l2,
                     int n_slots, int n_used, int n_rows, float* lb, float* best, int first, hipStream_t s,
                     int* improved = nullptr);
// joint optimisation of intermediate bounds (Sec. 3.3, Eq. opt_non_convex);
// current bounds lcur / ucur and root bounds are [B][nd] (one row per subdomain)
// status / chord of columns [0, nd_x) of a handle (row stride nd_x) from the
// current bounds; status0 holds the handle's words at the root bounds
void launch_joint_refresh(uint32_t* status, const uint32_t* status0, float2* chord, const float* lcur,
                          const float* ucur, int B, int nd_x, int nd, hipStream_t s);
// shared alpha' [B][2][uc_b] at CROWN's slope of each subdomain's root bounds
void launch_joint_alpha_init(float* ash, const int* ulist, const int64_t* uoff, const Batch& bt, int B, int d,
                             hipStream_t s);
// layer (off, d) bounds from an intermediate pass's rows [B][2d] (lower
// bounds of z, then of -z), clipped by the root bounds; ml / mu = 1 where the
// gradient follows the computed bound (not looser than the root's by more
// than a relative 1e-4)
void launch_joint_clip(const float* lb, int d, int off, const float* lroot, const float* uroot, float* lcur,
                       float* ucur, uint8_t* ml, uint8_t* mu, int B, int nd, hipStream_t s);
// shared alpha' [B][2][uc_b] / beta' [nnz][2] copied to every row of their
// side (rows k >= d hold the upper bounds) in the pass's own layouts
void launch_joint_bcast(float* arow, const float* ash, float* brow, const float* bsh, const Batch& bt, int d,
                        int64_t nnz, hipStream_t s);
// shared gradients = per side, sum over its rows of w[row] x the row's gradient
void launch_joint_reduce(float* gash, const float* garow, float* gbsh, const float* gbrow, const float* w,
                         const Batch& bt, int B, int d, int64_t nnz, hipStream_t s);
// dL, dU [B][nd] += d(sum_rows w g)/dl, /du at the unstable neurons of columns
// [col0, nd_x) of a handle (w null: every row weighs 1), from its stored A
// (acomp) and the adjoint's zbar at upper-chord neurons (zchord)
void launch_joint_cot(float* dL, float* dU, const uint32_t* status, const float* acomp, const float* zchord,
                      const float* w, const float* lcur, const float* ucur, const Batch& bt, int col0, int nd_x,
                      int nd, int B, hipStream_t s);
// row weights of layer (off, d)'s pass: dL where ml (lower rows), -dU where mu
// (upper rows), else 0
void launch_joint_weights(float* w, const float* dL, const float* dU, const uint8_t* ml, const uint8_t* mu, int B,
                          int d, int off, int nd, hipStream_t s);
// copy the variables of the rows flagged in improved into abest / bbest
void launch_keep_best(const float* alpha, const float* beta, float* abest, float* bbest, const int* improved,
                      const Batch& bt, hipStream_t s);
// the split neurons' Adam steps a conv layer's adjoint deferred (Vars::gsplit):
// every split t in a column flagged in defer [nd], every spec row
void launch_split_adam(const Batch& bt, const Vars& v, const int* split_dom, const int* split_col,
                       const uint8_t* defer, int64_t nnz, hipStream_t s);
void launch_adam(float* x, const float* g, float* m1, float* m2, int64_t n, float lr, float bc1, float bc2,
                 float lo, float hi, hipStream_t s);
void launch_fill(float* p, float v, int64_t n, hipStream_t s);
void launch_alpha_default(float* alpha, const int* ulist, const int64_t* uoff, const Batch& bt, hipStream_t s);

}  // namespace cvb
