// Device-side shared definitions of libcvbound (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cvb {

constexpr int kWave = 64;

// Per (subdomain, neuron) status record, 32 bits.  Bits 31..30: kind, the
// cases of Eq. definition_D (l >= 0 active, u <= 0 inactive, otherwise
// unstable) with split neurons as a fourth kind.  UNSTABLE: bits 29..0 hold
// the neuron's index in its property's unstable list (its alpha entry is
// row base + that index).  SPLIT: bit 29 is the side (1: z >= 0, set Z+) and
// bits 28..0 the split's index in the CSR split arrays (its beta row).
constexpr uint32_t kInactive = 0u << 30;
constexpr uint32_t kActive = 1u << 30;
constexpr uint32_t kUnstable = 2u << 30;
constexpr uint32_t kSplit = 3u << 30;
constexpr uint32_t kKindMask = 3u << 30;
constexpr uint32_t kCidxMask = (1u << 30) - 1;
constexpr uint32_t kSidePos = 1u << 29;
constexpr uint32_t kSplitMask = (1u << 29) - 1;
constexpr int64_t kMaxSplits = (int64_t)1 << 29;

// Everything a kernel needs to know about the batch, by value.
struct Batch {
  int m;          // specification rows per subdomain
  int n_rows;     // B * m
  int nd;         // sum of ReLU-layer widths
  int d0;         // input width
  int w64;        // 64-bit words per row of the x* sign planes
  const int* prop;          // [B] property of each subdomain
  const int64_t* aoff;      // [B] first alpha entry of each subdomain
  const int64_t* rbase;     // [n_rows] first alpha entry of each row
  const int* ucount;        // [P] root-unstable neurons per property
  const int64_t* sptr;      // [B+1] CSR offsets of each subdomain's splits
  const uint32_t* status;   // [B, nd] status records
  const int* cidx;          // [P, nd] index in the property's unstable list or -1
  const float2* chord;      // [P, nd] (u/(u-l), -u l/(u-l)) for unstable neurons
  const float* adef;        // [P, nd] default alpha (used when a pass has no alpha array)
  const float* xlo;         // [P, d0]
  const float* xhi;         // [P, d0]
  // sound mode (null sw otherwise): weight of |Lambda_k| in each row's bound
  // on the float32 rounding error, and the weight sg of every term of the
  // constant and of the concretisation
  const float* sw;          // [P, nd]
  float sg;
  // l2-ball input sets (null l2x0: the box x_lo, x_hi): centre and radius of
  // each property's ball (the q = 2 form of Eq. beta_crown_lp)
  const float* l2x0;        // [P, d0]
  const float* l2eps;       // [P]
  // dual exponent q = p/(p-1) of the l_p ball (2 for the l2 ball); read only
  // with l2x0 set
  float lpq;
};

// Variables of one pass.
struct Vars {
  const float* alpha;  // [n_alpha]
  const float* beta;   // [nnz, m]
  float* acomp;        // [n_alpha] A at unstable neurons, written in grad passes (or null)
  float* galpha;       // [n_alpha] gradient out (fwd passes)
  float* gbeta;        // [nnz, m]
  uint64_t* xpos;      // [n_rows, w64] bit set where A(0) > 0 (convolution first layer)
  uint64_t* xneg;      // [n_rows, w64] bit set where A(0) < 0
  float* xdense;       // [n_rows, ldx] the box minimiser x* itself (dense first layer)
  int ldx;
  // l2-ball adjoint: eps / ||A(0)||_2 of each row (x* = x0 - l2s A(0)), or null
  const float* l2s;
  // joint optimisation of intermediate bounds: where an unstable neuron's
  // stored A is negative (upper chord), the adjoint's zbar there, in the
  // neuron's alpha slot (the gradient of the bound in l and u needs it), or null
  float* zchord;
  // The network's own forward pass at x* (upper bound) instead of the
  // adjoint's relaxed one: when set, the forward kernels apply the exact ReLU
  // and clear sat[row] where a pre-activation breaks a split of the row's
  // subdomain.
  int* sat;
  // Projected Adam fused into the adjoint (optimisation passes): when adam is
  // set, each gradient entry is applied in place by its owning (row, neuron)
  // instead of being written to galpha / gbeta.  alpha_w / beta_w alias alpha /
  // beta; every entry has exactly one owner, which reads it before writing it.
  int adam;
  float lr_a, lr_b, bc1, bc2;
  float* alpha_w;
  float* beta_w;
  float* ma;
  float* va;
  float* mb;
  float* vb;
  // With adam set, a conv layer's adjoint may leave its split neurons' steps
  // to split_adam_k after the pass (their variables' reads would otherwise
  // wait inside the epilogue): it writes each split neuron's beta gradient
  // here ([nnz, m]) and touches neither variable.
  float* gsplit;
};

// The exact ReLU of the network at x* (the primal side of Alg. 1): clears
// *sat_row when zb breaks the split of a split neuron (z >= 0 for a z >= 0
// split, z <= 0 for a z < 0 split: the strict side closed, as in the LP).
// Several lanes may clear the same flag; they all store the same 0.
__device__ __forceinline__ float true_relu(uint32_t rec, float zb, int* sat_row) {
  if ((rec & kKindMask) == kSplit) {
    const bool pos = (rec & kSidePos) != 0;
    if (pos ? zb < 0.f : zb > 0.f) *sat_row = 0;
  }
  return fmaxf(zb, 0.f);
}

// One projected Adam ascent step (Kingma & Ba: beta1 0.9, beta2 0.999, eps
// 1e-8; bc1 = 1 - 0.9^t, bc2 = 1 - 0.999^t), clamped to [lo, hi], from an
// entry's value xv, moments m1v, m2v and gradient g: the new moments in a, b
// and the new value returned.
__device__ __forceinline__ float adam_values(float g, float lr, float bc1, float bc2, float lo, float hi, float xv,
                                             float m1v, float m2v, float& a, float& b) {
  // fmaf keeps the products with the moments next to g: a product of a moment
  // alone would be hoisted to where the moment is read ahead, stalling there
  a = fmaf(0.9f, m1v, 0.1f * g);
  b = fmaf(0.999f, m2v, 0.001f * g * g);
  // bias corrections as reciprocals (uniform across the launch); the square
  // root and the reciprocal are the hardware's single instructions (each
  // within 1 ulp; the correctly rounded library forms cost some 25 more
  // instructions per entry): within a few ulp of
  // lr (a / bc1) / (sqrt(b / bc2) + 1e-8)
  const float den = __builtin_amdgcn_sqrtf(b * (1.f / bc2)) + 1e-8f;
  const float step = lr * a * (1.f / bc1) * __builtin_amdgcn_rcpf(den);
  return fminf(fmaxf(xv + step, lo), hi);
}

// The step on entry i of x (moments m1, m2): adam_step takes the entry's
// current value and moments as arguments (read ahead by the caller);
// adam_apply reads them itself.
__device__ __forceinline__ float adam_step(float* x, float* m1, float* m2, int64_t i, float g, float lr, float bc1,
                                           float bc2, float lo, float hi, float xv, float m1v, float m2v) {
  float a, b;
  const float xn = adam_values(g, lr, bc1, bc2, lo, hi, xv, m1v, m2v, a, b);
  m1[i] = a;
  m2[i] = b;
  x[i] = xn;
  return xn;
}

__device__ __forceinline__ float adam_apply(float* x, float* m1, float* m2, int64_t i, float g, float lr, float bc1,
                                            float bc2, float lo, float hi) {
  return adam_step(x, m1, m2, i, g, lr, bc1, bc2, lo, hi, x[i], m1[i], m2[i]);
}

// Per-launch epilogue parameters (one layer).
struct Epi {
  int layer_off;       // offset of the output layer in the nd axis
  int n;               // output width
  const float* bias;   // [n] bias of that layer (fwd: added to z; bwd: b of the relaxed layer)
  float* out;          // [n_rows, ldo] next operand
  int ldo;
  float* part;         // [n_slots, n_rows] partial constants (slot-major)
  float* perr;         // [n_slots, n_rows] partial rounding-error bounds (sound mode), or null
  float* psq;          // [n_slots, n_rows] partial sums of A(0)^2 (l2 ball), or null
  // first layer of the l2-ball adjoint: W(1) x0 + b(1) per property [P, n];
  // zbar(1) = wx0 - l2s[row] (W(1) A(0)) then replaces W(1) x* + b(1)
  const float* wx0;
  int n_slots;
  int slot0;           // first slot of this launch
  // The adjoint's top ReLU layer inside the optimiser (null top_out
  // otherwise): after the Adam step the epilogue also relaxes the next
  // iteration's A(L-1) = C_p W(L) with the new variables -- the top layer of
  // the next back-substitution -- writing Lambda(L-1) to top_out and its
  // constant into slots slot0 + column tile (tile 0 adds C_p b(L)).
  float* top_out;
  const float* cw;     // [P, m, ldcw] C_p W(L)
  int64_t cw_pstride;
  int ldcw;
  const float* cb;     // [P, m] C_p b(L)
  int64_t cb_pstride;
};

struct RowInfo {
  int b, k, p;
  int64_t abase;  // alpha index of (b, k, unstable #0)
};

__device__ __forceinline__ RowInfo row_info(const Batch& bt, int r) {
  RowInfo ri;
  ri.b = r / bt.m;
  ri.k = r - ri.b * bt.m;
  ri.p = bt.prop[ri.b];
  ri.abase = bt.rbase[r];
  return ri;
}

// Relaxation of one neuron of a ReLU layer during back-substitution (Lemma
// 2.1 cases of Eq. definition_D / definition_lowerb, plus the split term
// beta^T S of Eq. definition_A).  a = A(i)_j.  Returns Lambda(i)_j and adds
// A lowerb + Lambda b to *cst.  Stores a into acomp at unstable neurons when
// acomp is set (the adjoint needs the branch and the value).
__device__ __forceinline__ float relax_value(const Batch& bt, const Vars& v, const RowInfo& ri, uint32_t rec,
                                             float2 ch, float coef, float a, float bias, float* cst) {
  // written as selects (no divergent branches); the same operations as the
  // case analysis: active a, inactive 0, unstable alpha a (a >= 0) or the
  // chord a u/(u-l) with a (-ul/(u-l)) into the constant, split a - beta
  // (z >= 0: D = 1, S = -1) or beta (z < 0: D = 0, S = +1); coef is alpha
  // for an unstable neuron and beta for a split one
  const uint32_t kind = rec & kKindMask;
  const bool uns = kind == kUnstable;
  const bool neg = uns && !(a >= 0.f);
  float lam = kind == kActive ? a : 0.f;
  lam = uns ? (neg ? a * ch.x : coef * a) : lam;
  lam = kind == kSplit ? ((rec & kSidePos) ? a - coef : coef) : lam;
  *cst = neg ? fmaf(a, ch.y, *cst) : *cst;
  *cst = fmaf(lam, bias, *cst);
  return lam;
}

// The variables that multiply neuron (row, col): alpha for an unstable
// neuron, beta for a split one, each read into a register of its own (two
// loads into one register from the two sides of a divergent branch would
// make the second wait for every load in flight).
__device__ __forceinline__ void relax_vars(const Batch& bt, const Vars& v, const RowInfo& ri, uint32_t rec, int64_t pc,
                                           float* al, float* be) {
  const uint32_t kind = rec & kKindMask;
  *al = 0.f;
  *be = 0.f;
  if (kind == kUnstable) {
    const int64_t ai = ri.abase + (rec & kCidxMask);
    *al = v.alpha ? v.alpha[ai] : bt.adef[pc];
  }
  if (kind == kSplit) *be = v.beta[(int64_t)(rec & kSplitMask) * bt.m + ri.k];
}

__device__ __forceinline__ float relax_pick(uint32_t rec, float al, float be) {
  return (rec & kKindMask) == kSplit ? be : al;
}

// (sound mode: also adds |Lambda| sw of the neuron to *err)
__device__ __forceinline__ float relax_bwd(const Batch& bt, const Vars& v, const RowInfo& ri, int layer_off,
                                          int j, float a, float bias, float* cst, float* err) {
  const int col = layer_off + j;
  const uint32_t rec = bt.status[(int64_t)ri.b * bt.nd + col];
  const int64_t pc = (int64_t)ri.p * bt.nd + col;
  const float2 ch = bt.chord[pc];
  if (v.acomp && (rec & kKindMask) == kUnstable) v.acomp[ri.abase + (rec & kCidxMask)] = a;
  float al, be;
  relax_vars(bt, v, ri, rec, pc, &al, &be);
  const float lam = relax_value(bt, v, ri, rec, ch, relax_pick(rec, al, be), a, bias, cst);
  if (bt.sw) *err = fmaf(fabsf(lam), bt.sw[pc], *err);
  return lam;
}

// Box minimiser contribution min(a xl, a xu) (Eq. beta_crown_lp for a box).
__device__ __forceinline__ float conc_term(float a, float xl, float xu) {
  return fminf(a * xl, a * xu);
}

// One entry a of A(0) over an l_p ball (Eq. beta_crown_lp with the dual
// exponent q): adds |a|^q to the row's q-norm sum and returns
// sign(a) |a|^(q-1), the direction of the minimiser
// x* = x0 - eps sign(A(0)) |A(0)|^(q-1) / ||A(0)||_q^(q-1) (Hoelder's
// equality case).  q = 2: a*a (fused) and a itself.  Otherwise the power is
// formed as 2^((q-1) log2 |a|).
__device__ __forceinline__ float lp_entry(float a, float q, float* sum) {
  if (q == 2.f) {
    *sum = fmaf(a, a, *sum);
    return a;
  }
  const float aa = fabsf(a);
  const float t = aa > 0.f ? exp2f((q - 1.f) * log2f(aa)) : 0.f;
  *sum = fmaf(aa, t, *sum);
  return copysignf(t, a);
}

// x* of the box minimum: xl where A(0) > 0, xu where < 0, the centre at 0.
__device__ __forceinline__ float xstar(bool pos, bool neg, float xl, float xu) {
  return pos ? xl : (neg ? xu : 0.5f * (xl + xu));
}

// Adjoint at one neuron of ReLU layer i during the forward sweep: zb =
// zbar(i)_j (bias included).  Writes the gradient of alpha / beta owned by
// this (row, neuron) -- or applies the fused Adam step -- and returns
// zhat(i)_j = D zbar + lowerb.  a_st is the stored A(i)_j and al the alpha of
// an unstable neuron; be is the beta of a split neuron.
// With mom_ahead, mom holds the Adam moments of an unstable neuron's alpha,
// read ahead by the caller together with al (its current value).  var_new,
// when set, receives the neuron's variable after this step (alpha of an
// unstable neuron, beta of a split one).
// kZchord = false compiles the zchord store out (kernels that never run in a
// pass of the joint optimisation, where registers are tight).
template <bool kZchord = true>
__device__ __forceinline__ float relax_fwd_value(const Batch& bt, const Vars& v, const RowInfo& ri, uint32_t rec,
                                                 float2 ch, float a_st, float al, int64_t pc, float zb,
                                                 bool mom_ahead = false, float2 mom = float2{0.f, 0.f},
                                                 float* var_new = nullptr) {
  const uint32_t kind = rec & kKindMask;
  if (kind == kActive) return zb;
  if (kind == kInactive) return 0.f;
  if (kind == kUnstable) {
    const int64_t ai = ri.abase + (rec & kCidxMask);
    float zh, g;
    if (a_st >= 0.f) {
      g = zb * a_st;
      zh = al * zb;
    } else {
      g = 0.f;
      zh = fmaf(ch.x, zb, ch.y);
      if (kZchord && v.zchord) v.zchord[ai] = zb;
    }
    float an = al;
    if (v.adam && mom_ahead) an = adam_step(v.alpha_w, v.ma, v.va, ai, g, v.lr_a, v.bc1, v.bc2, 0.f, 1.f, al, mom.x, mom.y);
    else if (v.adam) an = adam_apply(v.alpha_w, v.ma, v.va, ai, g, v.lr_a, v.bc1, v.bc2, 0.f, 1.f);
    else v.galpha[ai] = g;
    if (var_new) *var_new = an;
    return zh;
  }
  const bool pos = (rec & kSidePos) != 0;
  const int64_t bi = (int64_t)(rec & kSplitMask) * bt.m + ri.k;
  // a split neuron is root-unstable, so it owns an alpha entry: its gradient is 0
  const int64_t ai = ri.abase + bt.cidx[pc];
  const float gb = pos ? -zb : zb;
  if (v.gsplit) {  // (no var_new: the passes that defer never ask for it)
    v.gsplit[bi] = gb;
  } else if (v.adam) {
    const float bn = adam_apply(v.beta_w, v.mb, v.vb, bi, gb, v.lr_b, v.bc1, v.bc2, 0.f, INFINITY);
    adam_apply(v.alpha_w, v.ma, v.va, ai, 0.f, v.lr_a, v.bc1, v.bc2, 0.f, 1.f);
    if (var_new) *var_new = bn;
  } else {
    v.gbeta[bi] = gb;
    v.galpha[ai] = 0.f;
  }
  return pos ? zb : 0.f;
}

__device__ __forceinline__ float relax_fwd(const Batch& bt, const Vars& v, const RowInfo& ri, int layer_off,
                                          int j, float zb) {
  const int col = layer_off + j;
  const uint32_t rec = bt.status[(int64_t)ri.b * bt.nd + col];
  const int64_t pc = (int64_t)ri.p * bt.nd + col;
  const float2 ch = bt.chord[pc];
  float a_st = 0.f, al = 0.f;
  if ((rec & kKindMask) == kUnstable) {
    const int64_t ai = ri.abase + (rec & kCidxMask);
    a_st = v.acomp[ai];
    al = v.alpha ? v.alpha[ai] : bt.adef[pc];
  }
  return relax_fwd_value(bt, v, ri, rec, ch, a_st, al, pc, zb);
}

// Butterfly sums by DPP moves within rows of 16 lanes (no LDS round trip).
// Each step adds the values of lanes l and l ^ o; once the lanes of a quad
// (of a half row) hold equal values, the half-row (row) mirror pairs every
// lane with one of the partner group, so the additions, and with them the
// roundings, are those of the xor butterfly (float addition commutes).
template <int kCtrl>
__device__ __forceinline__ float dpp_step(float x) {
  return x + __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), kCtrl, 0xF, 0xF, true));
}

__device__ __forceinline__ float wave_sum16(float x) {
  // sum over the 16 lanes that share lane/16 (xor 1, 2, 4, 8)
  x = dpp_step<0xB1>(x);   // quad_perm [1, 0, 3, 2]: lane ^ 1
  x = dpp_step<0x4E>(x);   // quad_perm [2, 3, 0, 1]: lane ^ 2
  x = dpp_step<0x141>(x);  // row_half_mirror: the other quad of the half row
  x = dpp_step<0x140>(x);  // row_mirror: the other half of the row
  return x;
}

__device__ __forceinline__ float wave_sum(float x) {
  // the row sums, then xor 16 and xor 32 across rows as
  // (r0 + r1) + (r2 + r3) in every lane
  x = wave_sum16(x);
  const float r0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 0));
  const float r1 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 16));
  const float r2 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 32));
  const float r3 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 48));
  return (r0 + r1) + (r2 + r3);
}

}  // namespace cvb
