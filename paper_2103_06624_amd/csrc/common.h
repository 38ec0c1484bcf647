// Device-side shared definitions of libcvbound (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cvb {

constexpr int kWave = 64;

// Per (subdomain, neuron) status word.  Bits 15..14: kind.  For SPLIT, bit 13
// is the side (1: z >= 0, set Z+) and bits 12..0 the split's position in the
// subdomain's CSR list.  Root kinds follow the cases of Eq. definition_D:
// l >= 0 active, u <= 0 inactive, otherwise unstable.
constexpr uint16_t kInactive = 0u << 14;
constexpr uint16_t kActive = 1u << 14;
constexpr uint16_t kUnstable = 2u << 14;
constexpr uint16_t kSplit = 3u << 14;
constexpr uint16_t kKindMask = 3u << 14;
constexpr uint16_t kSidePos = 1u << 13;
constexpr uint16_t kSlotMask = (1u << 13) - 1;
constexpr int kMaxDepth = (1 << 13) - 1;

// Everything a kernel needs to know about the batch, by value.
struct Batch {
  int m;          // specification rows per subdomain
  int n_rows;     // B * m
  int nd;         // sum of ReLU-layer widths
  int d0;         // input width
  int w64;        // 64-bit words per row of the x* sign planes
  const int* prop;          // [B] property of each subdomain
  const int64_t* aoff;      // [B] first alpha entry of each subdomain
  const int* ucount;        // [P] root-unstable neurons per property
  const int64_t* sptr;      // [B+1] CSR split offsets
  const uint16_t* status;   // [B, nd]
  const int* cidx;          // [P, nd] index in the property's unstable list or -1
  const float2* chord;      // [P, nd] (u/(u-l), -u l/(u-l)) for unstable neurons
  const float* adef;        // [P, nd] default alpha (used when a pass has no alpha array)
  const float* xlo;         // [P, d0]
  const float* xhi;         // [P, d0]
};

// Variables of one pass.
struct Vars {
  const float* alpha;  // [n_alpha]
  const float* beta;   // [nnz, m]
  float* acomp;        // [n_alpha] A at unstable neurons, written in grad passes (or null)
  float* galpha;       // [n_alpha] gradient out (fwd passes)
  float* gbeta;        // [nnz, m]
  uint64_t* xpos;      // [n_rows, w64] bit set where A(0) > 0
  uint64_t* xneg;      // [n_rows, w64] bit set where A(0) < 0
};

// Per-launch epilogue parameters (one layer).
struct Epi {
  int layer_off;       // offset of the output layer in the nd axis
  int n;               // output width
  const float* bias;   // [n] bias of that layer (fwd: added to z; bwd: b of the relaxed layer)
  float* out;          // [n_rows, ldo] next operand
  int ldo;
  float* part;         // [n_rows, n_slots] partial constants
  int n_slots;
  int slot0;           // first slot of this launch
};

struct RowInfo {
  int b, k, p;
  int64_t abase;  // alpha index of (b, k, unstable #0)
  int64_t sbase;  // first split of b
};

__device__ __forceinline__ RowInfo row_info(const Batch& bt, int r) {
  RowInfo ri;
  ri.b = r / bt.m;
  ri.k = r - ri.b * bt.m;
  ri.p = bt.prop[ri.b];
  ri.abase = bt.aoff[ri.b] + (int64_t)ri.k * bt.ucount[ri.p];
  ri.sbase = bt.sptr[ri.b];
  return ri;
}

// Relaxation of one neuron of a ReLU layer during back-substitution (Lemma
// 2.1 cases of Eq. definition_D / definition_lowerb, plus the split term
// beta^T S of Eq. definition_A).  a = A(i)_j.  Returns Lambda(i)_j and adds
// A lowerb + Lambda b to *cst.  Stores a into acomp at unstable neurons when
// acomp is set (the adjoint needs the branch and the value).
__device__ __forceinline__ float relax_bwd(const Batch& bt, const Vars& v, const RowInfo& ri, int layer_off,
                                          int j, float a, float bias, float* cst) {
  const int col = layer_off + j;
  const uint16_t st = bt.status[(int64_t)ri.b * bt.nd + col];
  const uint16_t kind = st & kKindMask;
  float lam;
  if (kind == kActive) {
    lam = a;
  } else if (kind == kInactive) {
    lam = 0.f;
  } else if (kind == kUnstable) {
    const int64_t pc = (int64_t)ri.p * bt.nd + col;
    const int64_t ai = ri.abase + bt.cidx[pc];
    if (v.acomp) v.acomp[ai] = a;
    if (a >= 0.f) {
      lam = (v.alpha ? v.alpha[ai] : bt.adef[pc]) * a;
    } else {
      const float2 ch = bt.chord[pc];
      lam = a * ch.x;
      *cst = fmaf(a, ch.y, *cst);
    }
  } else {
    const bool pos = (st & kSidePos) != 0;
    const float be = v.beta[(ri.sbase + (st & kSlotMask)) * bt.m + ri.k];
    lam = pos ? a - be : be;  // D = 1, S = -1 for z >= 0; D = 0, S = +1 for z < 0
  }
  *cst = fmaf(lam, bias, *cst);
  return lam;
}

// Box minimiser contribution min(a xl, a xu) (Eq. beta_crown_lp for a box).
__device__ __forceinline__ float conc_term(float a, float xl, float xu) {
  return fminf(a * xl, a * xu);
}

// x* of the box minimum: xl where A(0) > 0, xu where < 0, the centre at 0.
__device__ __forceinline__ float xstar(bool pos, bool neg, float xl, float xu) {
  return pos ? xl : (neg ? xu : 0.5f * (xl + xu));
}

// Adjoint at one neuron of ReLU layer i during the forward sweep: zb =
// zbar(i)_j (bias included).  Writes the gradient of alpha / beta owned by
// this (row, neuron) and returns zhat(i)_j = D zbar + lowerb.
__device__ __forceinline__ float relax_fwd(const Batch& bt, const Vars& v, const RowInfo& ri, int layer_off,
                                          int j, float zb) {
  const int col = layer_off + j;
  const uint16_t st = bt.status[(int64_t)ri.b * bt.nd + col];
  const uint16_t kind = st & kKindMask;
  if (kind == kActive) return zb;
  if (kind == kInactive) return 0.f;
  if (kind == kUnstable) {
    const int64_t pc = (int64_t)ri.p * bt.nd + col;
    const int64_t ai = ri.abase + bt.cidx[pc];
    const float a = v.acomp[ai];
    if (a >= 0.f) {
      v.galpha[ai] = zb * a;
      return (v.alpha ? v.alpha[ai] : bt.adef[pc]) * zb;
    }
    v.galpha[ai] = 0.f;
    const float2 ch = bt.chord[pc];
    return fmaf(ch.x, zb, ch.y);
  }
  const bool pos = (st & kSidePos) != 0;
  v.gbeta[(ri.sbase + (st & kSlotMask)) * bt.m + ri.k] = pos ? -zb : zb;
  // a split neuron is root-unstable, so it owns an alpha entry: its gradient is 0
  const int64_t pc = (int64_t)ri.p * bt.nd + col;
  v.galpha[ri.abase + bt.cidx[pc]] = 0.f;
  return pos ? zb : 0.f;
}

__device__ __forceinline__ float wave_sum16(float x) {
  // sum over the 16 lanes that share lane/16 (xor within 16-lane groups)
  x += __shfl_xor(x, 1, 64);
  x += __shfl_xor(x, 2, 64);
  x += __shfl_xor(x, 4, 64);
  x += __shfl_xor(x, 8, 64);
  return x;
}

__device__ __forceinline__ float wave_sum(float x) {
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

}  // namespace cvb
