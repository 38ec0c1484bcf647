// Fused chains of dense layers (gfx950, FP32 MFMA).
//
// One workgroup of 8 waves owns a contiguous block of rows (subdomain x spec
// row) and carries it through a run of consecutive dense layers without
// leaving the chip: the current Lambda (back-substitution) or zhat (adjoint)
// of its rows lives in LDS, and each layer's weights stream through a ring of
// LDS slabs.
//
//   chain_bwd: top ReLU layer (relaxation of A(L-1) = C W(L), Sec. 2.1 /
//     Lemma 2.1) -> A(i-1) = Lambda(i) W(i) for i = L-1 .. lo (Eq.
//     definition_A), each followed by the next layer's relaxation; the last
//     step concretises over the box (Eq. beta_crown_lp) or writes the relaxed
//     Lambda(lo-1) to HBM for a convolution layer below.
//   chain_fwd: zbar(i) = W(i) zhat(i-1) + b(i) for i = lo .. L-1, zhat(lo-1)
//     read from HBM, with the adjoint's gradients (or the fused Adam step).
//
// Work split.  The rows of the batch are divided evenly over the grid (one
// workgroup per compute unit), so every CU carries the same load; a
// workgroup's rows are padded to 16-row MFMA blocks (RB blocks).  Per layer
// the output is a grid of 16x16 units (row block, column block); the 8 waves
// take contiguous runs of units in column-major order, so each wave reuses
// its A fragments across the row blocks and the runs differ by at most one
// unit.
//
// Weight pipeline.  The layer's weights (K-contiguous rows, zero-padded) are
// read 16 k at a time for the chunk's columns by all 512 threads, each slab
// loaded two steps ahead into registers and parked in a 3-slot LDS ring one
// step ahead, with one barrier per step.  MFMA 16x16x4 f32: each lane reads 4
// consecutive k of its row (A from the LDS-resident rows, B from the slab)
// with one b128 read and feeds them to 4 MFMAs (k slot g of MFMA t holds
// k = 4g + t for both operands, so the products pair up).
//
// Per-neuron phases (relaxation, adjoint step, concretisation) give each row
// TPR consecutive threads; a thread takes every TPR-th neuron and issues the
// loads of E neurons together (status record, chord, bias, then the alpha /
// beta they select), so a whole batch's gathers are in flight at once.
#include <algorithm>

#include "common.h"
#include "internal.h"

typedef float floatx4 __attribute__((ext_vector_type(4)));

namespace cvb {

namespace {

constexpr int kCT = 512;     // threads per workgroup
constexpr int KS = 32;       // k per pipeline step (two 16-k MFMA sub-steps)
constexpr int WLD = KS + 4;  // LDS pitch of a weight-slab row (floats): conflict-free b128 reads
constexpr int NSTAGE = 2;    // slabs resident in LDS
constexpr int SLAB4 = 4;     // float4 per thread per slab: 256 columns x 8 / 512 threads
constexpr int kWidth = 256;  // widest LDS-resident layer

template <int RB>
struct Geo {
  static constexpr int T = 16 * RB;                     // row capacity
  static constexpr int TPR = kCT / T;                   // threads per row in the per-neuron phases
  static constexpr int E = (kWidth + TPR - 1) / TPR;    // neurons per thread: one batch covers a row
};

// Slab s of the chunk's weights: columns [c0, c0 + nc) x k [32 s, 32 s + 32),
// one float4 per (column, eighth) over the 512 threads (nc <= 256), four per
// thread.  Rows are zero-padded to 16-multiples and k to 32-multiples, so
// every read is in bounds and the padding contributes zeros.  The loads are
// unconditional (indices clamped: threads past the slab repeat its last
// float4) so that neither they nor the LDS stores need a per-lane predicate.
struct Slab4 {
  float4 v[SLAB4];
};

__device__ __forceinline__ Slab4 wload(const ChainLayer& L, int c0, int nc, int s, int nks) {
  const int sc = min(s, nks - 1);
  Slab4 r;
#pragma unroll
  for (int i = 0; i < SLAB4; ++i) {
    const int f = min((int)threadIdx.x + kCT * i, nc * 8 - 1);
    r.v[i] = *reinterpret_cast<const float4*>(L.Bt + (int64_t)(c0 + (f >> 3)) * L.ldb + sc * KS + (f & 7) * 4);
  }
  return r;
}

__device__ __forceinline__ void wstore(float* ring, int np, int nc, int s, int nks, const Slab4& st) {
  if (s >= nks) return;  // uniform
  float* slab = ring + (s % NSTAGE) * np * WLD;
#pragma unroll
  for (int i = 0; i < SLAB4; ++i) {
    const int f = min((int)threadIdx.x + kCT * i, nc * 8 - 1);
    *reinterpret_cast<float4*>(slab + (f >> 3) * WLD + (f & 7) * 4) = st.v[i];
  }
}

// Units of this wave: [u0, u0 + UW), unit u = column block u / RB, row block
// u % RB; every wave takes UW units (UW = ceil(units / 8)), those past the
// chunk's units are dummies that multiply zeros and are not stored.
template <int UW>
__device__ __forceinline__ int wave_u0() {
  return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6) * UW;  // wave-uniform: scalar control flow
}

// Fragments of one 16-k step for a wave: A of the RB row blocks and B of the
// (at most 3) column blocks its run of units touches, in named registers (an
// array would be indexed through scratch).
struct Frags {
  float4 a0, a1, a2, b0, b1, b2;
};

// Fragments of the 16-k sub-step at column k of the resident rows and offset
// ks within the slab.
template <int RB>
__device__ __forceinline__ Frags frag_load(const float* lam, int ldk, const float* slab, int k, int ks, int cb0,
                                           int ncb) {
  const int lane = threadIdx.x & 63;
  const int l15 = lane & 15, kq = 4 * (lane >> 4);
  auto a = [&](int rb) { return *reinterpret_cast<const float4*>(lam + (rb * 16 + l15) * ldk + k + kq); };
  auto b = [&](int i) {
    return *reinterpret_cast<const float4*>(slab + (min(cb0 + i, ncb - 1) * 16 + l15) * WLD + ks + kq);
  };
  Frags f;
  f.a0 = a(0);
  f.a1 = RB > 1 ? a(1) : f.a0;
  f.a2 = RB > 2 ? a(2) : f.a0;
  f.b0 = b(0);
  f.b1 = b(1);
  f.b2 = b(2);
  return f;
}

// acc[g] += A(row block of unit u0+g) x B(its column block) over one step; the
// MFMAs run across the units for each k so consecutive ones are independent.
// Component-wise choice among three values (c is wave-uniform): plain
// selects, so the operands stay in registers.
__device__ __forceinline__ float4 pick3(int c, float4 x, float4 y, float4 z) {
  float4 r;
  r.x = c == 0 ? x.x : (c == 1 ? y.x : z.x);
  r.y = c == 0 ? x.y : (c == 1 ? y.y : z.y);
  r.z = c == 0 ? x.z : (c == 1 ? y.z : z.z);
  r.w = c == 0 ? x.w : (c == 1 ? y.w : z.w);
  return r;
}

template <int RB, int UW>
__device__ __forceinline__ void frag_mma(Frags f, int u0, int nunits, int cb0, floatx4 (&acc)[UW]) {
  float4 av[UW], bv[UW];
  const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
  for (int g = 0; g < UW; ++g) {
    const int u = u0 + g;
    const int cb = u / RB, rb = u - cb * RB, ci = cb - cb0;
    av[g] = pick3(rb, f.a0, f.a1, f.a2);
    bv[g] = u < nunits ? pick3(ci, f.b0, f.b1, f.b2) : z;
  }
#pragma unroll
  for (int g = 0; g < UW; ++g) acc[g] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[g].x, bv[g].x, acc[g], 0, 0, 0);
#pragma unroll
  for (int g = 0; g < UW; ++g) acc[g] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[g].y, bv[g].y, acc[g], 0, 0, 0);
#pragma unroll
  for (int g = 0; g < UW; ++g) acc[g] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[g].z, bv[g].z, acc[g], 0, 0, 0);
#pragma unroll
  for (int g = 0; g < UW; ++g) acc[g] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[g].w, bv[g].w, acc[g], 0, 0, 0);
}

// acc = lam (the tile's rows, K = L.K) x weights for columns [c0, c0 + nc).
// Starts and ends with the ring free; ends after a barrier, so lam may be
// overwritten next.  Step s (32 k): the weight slab s+1 is requested, then
// both sub-steps' fragments are read and their MFMAs run while it is in
// flight, then it is parked in the other ring slot (read during step s-1,
// before the barrier that ended it).  Each step's loads complete within the
// step, so no register state crosses the loop edge with a load in flight.
template <int RB, int UW>
__device__ __forceinline__ void mma_chunk(const ChainLayer& L, const float* lam, int ldk, float* ring, int np, int c0,
                                          int nc, floatx4 (&acc)[UW]) {
  const int u0 = wave_u0<UW>();
  const int ncb = nc >> 4, nunits = RB * ncb;
  const int cb0 = min(u0 / RB, ncb - 1);
#pragma unroll
  for (int g = 0; g < UW; ++g) acc[g] = floatx4{0.f, 0.f, 0.f, 0.f};
  const int nks = (L.K + KS - 1) / KS;
  Slab4 st = wload(L, c0, nc, 0, nks);
  wstore(ring, np, nc, 0, nks, st);
  __syncthreads();
  for (int s = 0; s < nks; ++s) {
    st = wload(L, c0, nc, s + 1, nks);
    const float* slab = ring + (s % NSTAGE) * np * WLD;
    const Frags f0 = frag_load<RB>(lam, ldk, slab, s * KS, 0, cb0, ncb);
    const Frags f1 = frag_load<RB>(lam, ldk, slab, s * KS + 16, 16, cb0, ncb);
    frag_mma<RB, UW>(f0, u0, nunits, cb0, acc);
    frag_mma<RB, UW>(f1, u0, nunits, cb0, acc);
    wstore(ring, np, nc, s + 1, nks, st);
    __syncthreads();
  }
}

// Raw unit results into dst[row][col - c0] (pitch ldd).
template <int RB, int UW>
__device__ __forceinline__ void store_units(const floatx4 (&acc)[UW], int nc, float* dst, int ldd) {
  const int lane = threadIdx.x & 63;
  const int rsub = 4 * (lane >> 4), csub = lane & 15;
  const int u0 = wave_u0<UW>(), nunits = RB * (nc >> 4);
#pragma unroll
  for (int g = 0; g < UW; ++g) {
    const int u = u0 + g;
    if (u >= nunits) break;  // uniform
    const int cb = u / RB, rb = u - cb * RB;
#pragma unroll
    for (int r = 0; r < 4; ++r) dst[(rb * 16 + rsub + r) * ldd + cb * 16 + csub] = acc[g][r];
  }
}

// Relaxation of one row's neurons j = sub, sub + TPR, ... < n of the ReLU layer
// at nd-offset `off`: Lambda = relax(src), constants into *cst, result to dst.
// src / dst may alias (in place in LDS).
template <int TPR, int E>
__device__ __forceinline__ void relax_phase(const ChainArgs& a, const RowInfo& ri, const float* src, float* dst,
                                            int n, int off, const float* bias, int sub, float* cst) {
  const uint32_t* st = a.bt.status + (int64_t)ri.b * a.bt.nd + off;
  const float2* chp = a.bt.chord + (int64_t)ri.p * a.bt.nd + off;
  for (int j0 = sub; j0 < n; j0 += TPR * E) {
    uint32_t rec[E];
    float2 ch[E];
    float av[E], bs[E], al[E], be[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int j = j0 + TPR * e;
      const bool ok = j < n;
      rec[e] = ok ? st[j] : kInactive;
      ch[e] = ok ? chp[j] : make_float2(0.f, 0.f);
      av[e] = ok ? src[j] : 0.f;
      bs[e] = ok ? bias[j] : 0.f;
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int64_t pc = (int64_t)ri.p * a.bt.nd + off + j0 + TPR * e;
      relax_vars(a.bt, a.v, ri, rec[e], pc, &al[e], &be[e]);
      if (a.v.acomp && (rec[e] & kKindMask) == kUnstable) a.v.acomp[ri.abase + (rec[e] & kCidxMask)] = av[e];
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int j = j0 + TPR * e;
      if (j < n) dst[j] = relax_value(a.bt, a.v, ri, rec[e], ch[e], relax_pick(rec[e], al[e], be[e]), av[e], bs[e], cst);
    }
  }
}

// Box concretisation of one row's chunk: columns col0 + 16 w + t for
// half-words w = sub, sub + TPR, ...; sign planes of A(0) stored 16 bits at a
// time (col0 is a 16-multiple).
template <int TPR>
__device__ __forceinline__ void conc_phase(const ChainArgs& a, const RowInfo& ri, int row, const float* src,
                                           int col0, int ncols, int n, int sub, float* cst) {
  const float* xl = a.bt.xlo + (int64_t)ri.p * a.bt.d0;
  const float* xu = a.bt.xhi + (int64_t)ri.p * a.bt.d0;
  const int nw = ncols >> 4;
  for (int w = sub; w < nw; w += TPR) {
    uint32_t bp = 0, bn = 0;
#pragma unroll
    for (int q = 0; q < 16; q += 8) {
      float av[8], l8[8], u8[8];
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const int c = col0 + 16 * w + q + t;
        const bool ok = c < n;
        av[t] = src[16 * w + q + t];
        l8[t] = ok ? xl[c] : 0.f;
        u8[t] = ok ? xu[c] : 0.f;
      }
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const int c = col0 + 16 * w + q + t;
        if (c < n) {
          *cst += conc_term(av[t], l8[t], u8[t]);
          bp |= (av[t] > 0.f ? 1u : 0u) << (q + t);
          bn |= (av[t] < 0.f ? 1u : 0u) << (q + t);
          if (a.v.xdense) a.v.xdense[(int64_t)row * a.v.ldx + c] = xstar(av[t] > 0.f, av[t] < 0.f, l8[t], u8[t]);
        }
      }
    }
    if (a.v.xpos) {
      reinterpret_cast<uint16_t*>(a.v.xpos + (int64_t)row * a.bt.w64)[(col0 >> 4) + w] = (uint16_t)bp;
      reinterpret_cast<uint16_t*>(a.v.xneg + (int64_t)row * a.bt.w64)[(col0 >> 4) + w] = (uint16_t)bn;
    }
  }
}

// Adjoint step of one row's neurons j = sub, sub + TPR, ... < n of ReLU layer
// `off`: zhat = D (zbar + b) + lowerb written in place; gradients or Adam.
template <int TPR, int E>
__device__ __forceinline__ void relax_fwd_phase(const ChainArgs& a, const RowInfo& ri, float* z, int n, int off,
                                                const float* bias, int sub, bool write) {
  const uint32_t* st = a.bt.status + (int64_t)ri.b * a.bt.nd + off;
  const float2* chp = a.bt.chord + (int64_t)ri.p * a.bt.nd + off;
  for (int j0 = sub; j0 < n; j0 += TPR * E) {
    uint32_t rec[E];
    float2 ch[E];
    float zb[E], ast[E], al[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int j = j0 + TPR * e;
      const bool ok = j < n;
      rec[e] = ok ? st[j] : kInactive;
      ch[e] = ok ? chp[j] : make_float2(0.f, 0.f);
      zb[e] = ok ? z[j] + bias[j] : 0.f;
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
      ast[e] = 0.f;
      al[e] = 0.f;
      if ((rec[e] & kKindMask) == kUnstable) {
        const int64_t ai = ri.abase + (rec[e] & kCidxMask);
        ast[e] = a.v.acomp[ai];
        al[e] = a.v.alpha ? a.v.alpha[ai] : a.bt.adef[(int64_t)ri.p * a.bt.nd + off + j0 + TPR * e];
      }
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int j = j0 + TPR * e;
      if (j < n) {
        const float zh = relax_fwd_value(a.bt, a.v, ri, rec[e], ch[e], ast[e], al[e],
                                         (int64_t)ri.p * a.bt.nd + off + j, zb[e]);
        if (write) z[j] = zh;
      }
    }
  }
}

// Rows [r0, r1) of this workgroup: the batch divided evenly over the grid.
__device__ __forceinline__ void tile_rows(int R, int* r0, int* r1) {
  *r0 = (int)((int64_t)blockIdx.x * R / gridDim.x);
  *r1 = (int)((int64_t)(blockIdx.x + 1) * R / gridDim.x);
}

template <int RB, int UW>
__global__ __launch_bounds__(kCT) void chain_bwd(ChainArgs a) {
  constexpr int T = Geo<RB>::T, TPR = Geo<RB>::TPR, E = Geo<RB>::E;
  extern __shared__ __attribute__((aligned(16))) float sm[];
  __shared__ RowInfo rinfo[T];
  float* lam = sm;
  float* ring = sm + T * a.ldk;
  const int tid = threadIdx.x;
  int r0, r1;
  tile_rows(a.bt.n_rows, &r0, &r1);
  const int nrow = r1 - r0;
  if (tid < nrow) rinfo[tid] = row_info(a.bt, r0 + tid);
  for (int t = tid; t < T * a.ldk; t += kCT) lam[t] = 0.f;
  __syncthreads();
  const int rl = tid / TPR, sub = tid - rl * TPR;
  const int row = r0 + rl;
  const bool rok = rl < nrow;
  RowInfo ri{};
  if (rok) ri = rinfo[rl];
  float cst = 0.f;

  // top ReLU layer: Lambda(L-1) = relax(C W(L)) into LDS
  if (rok)
    relax_phase<TPR, E>(a, ri, a.CW + ri.p * a.cw_pstride + (int64_t)ri.k * a.ldcw, lam + rl * a.ldk, a.n_top,
                     a.top_off, a.top_bias, sub, &cst);
  __syncthreads();

  floatx4 acc[UW];
  for (int s = 0; s < a.nl; ++s) {
    const ChainLayer L = a.ly[s];
    const int n16 = (L.N + 15) & ~15;
    if (s < a.nl - 1) {
      mma_chunk<RB, UW>(L, lam, a.ldk, ring, a.np, 0, n16, acc);
      store_units<RB, UW>(acc, n16, lam, a.ldk);
      __syncthreads();
      if (rok) relax_phase<TPR, E>(a, ri, lam + rl * a.ldk, lam + rl * a.ldk, L.N, L.out_off, L.bias, sub, &cst);
      __syncthreads();
    } else {
      // columns in chunks of ncw (a 16-multiple), staged through the ring
      for (int c0 = 0; c0 < n16; c0 += a.ncw) {
        const int nc = min(a.ncw, n16 - c0);
        mma_chunk<RB, UW>(L, lam, a.ldk, ring, a.np, c0, nc, acc);
        store_units<RB, UW>(acc, nc, ring, a.ldk);
        __syncthreads();
        if (rok) {
          if (a.conc)
            conc_phase<TPR>(a, ri, row, ring + rl * a.ldk, c0, nc, L.N, sub, &cst);
          else
            relax_phase<TPR, E>(a, ri, ring + rl * a.ldk, a.out + (int64_t)row * a.ldo + c0, min(nc, L.N - c0),
                             L.out_off + c0, L.bias + c0, sub, &cst);
        }
        __syncthreads();
      }
    }
  }

  // per-row constant: the row's TPR partial sums in a fixed order, plus the
  // specification bias
  float* red = ring;  // free after the last barrier
  if (rl < T) red[rl * TPR + sub] = cst;
  __syncthreads();
  if (sub == 0 && rok) {
    float tot = 0.f;
    for (int q = 0; q < TPR; ++q) tot += red[rl * TPR + q];
    tot += a.Cb[ri.p * a.cb_pstride + ri.k];
    if (a.final) {
      if (a.lb) a.lb[row] = tot;
      if (a.best) a.best[row] = a.first ? tot : fmaxf(a.best[row], tot);
    } else {
      a.part[(int64_t)a.slot * a.bt.n_rows + row] = tot;
    }
  }
}

template <int RB, int UW>
__global__ __launch_bounds__(kCT) void chain_fwd(ChainArgs a) {
  constexpr int T = Geo<RB>::T, TPR = Geo<RB>::TPR, E = Geo<RB>::E;
  extern __shared__ __attribute__((aligned(16))) float sm[];
  __shared__ RowInfo rinfo[T];
  float* lam = sm;
  float* ring = sm + T * a.ldk;
  const int tid = threadIdx.x;
  int r0, r1;
  tile_rows(a.bt.n_rows, &r0, &r1);
  const int nrow = r1 - r0;
  if (tid < nrow) rinfo[tid] = row_info(a.bt, r0 + tid);
  for (int t = tid; t < T * a.ldk; t += kCT) lam[t] = 0.f;
  __syncthreads();
  {
    // zhat(lo-1) of the tile's rows
    const int K = a.ly[0].K;
    for (int t = tid; t < nrow * K; t += kCT) {
      const int r = t / K, k = t - r * K;
      lam[r * a.ldk + k] = a.in[(int64_t)(r0 + r) * a.ldi + k];
    }
  }
  __syncthreads();
  const int rl = tid / TPR, sub = tid - rl * TPR;
  const bool rok = rl < nrow;
  RowInfo ri{};
  if (rok) ri = rinfo[rl];
  floatx4 acc[UW];
  for (int s = 0; s < a.nl; ++s) {
    const ChainLayer L = a.ly[s];
    const bool last = s == a.nl - 1;
    const int n16 = (L.N + 15) & ~15;
    mma_chunk<RB, UW>(L, lam, a.ldk, ring, a.np, 0, n16, acc);
    store_units<RB, UW>(acc, n16, lam, a.ldk);
    __syncthreads();
    if (rok) relax_fwd_phase<TPR, E>(a, ri, lam + rl * a.ldk, L.N, L.out_off, L.bias, sub, !last);
    __syncthreads();
  }
}

template <int RB, int UW>
void set_lds_limit(int bytes) {
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&chain_bwd<RB, UW>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&chain_fwd<RB, UW>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

template <bool BWD>
void launch_chain(const ChainArgs& a, hipStream_t s) {
  const size_t sm = chain_smem_bytes(a.rb, a.np);
  const int key = a.rb * 8 + a.uw;
#define CVB_CHAIN_CASE(R, U)                                  \
  case R * 8 + U:                                             \
    if (BWD) launch_k(chain_bwd<R, U>, a.grid, kCT, sm, s, a); \
    else launch_k(chain_fwd<R, U>, a.grid, kCT, sm, s, a);     \
    break;
  switch (key) {
    CVB_CHAIN_CASE(1, 1)
    CVB_CHAIN_CASE(1, 2)
    CVB_CHAIN_CASE(2, 1)
    CVB_CHAIN_CASE(2, 2)
    CVB_CHAIN_CASE(2, 3)
    CVB_CHAIN_CASE(2, 4)
    CVB_CHAIN_CASE(3, 1)
    CVB_CHAIN_CASE(3, 2)
    CVB_CHAIN_CASE(3, 3)
    CVB_CHAIN_CASE(3, 4)
    CVB_CHAIN_CASE(3, 5)
    CVB_CHAIN_CASE(3, 6)
    default: break;
  }
#undef CVB_CHAIN_CASE
}

}  // namespace

size_t chain_smem_bytes(int rb, int np) {
  const size_t ldk = (size_t)np + 4;
  const size_t lam = (size_t)16 * rb * ldk;
  const size_t ring = std::max((size_t)NSTAGE * np * WLD, lam + 32);
  return (lam + ring) * sizeof(float);
}

int chain_units_per_wave(int rb, int ncw) { return (rb * (ncw / 16) + 7) / 8; }

bool chain_units_fit(int rb, int np, int ncw) {
  return np % 32 == 0 && np <= kWidth && ncw % 16 == 0 && ncw <= np && rb >= 1 && rb <= kChainRowBlocks &&
         chain_units_per_wave(rb, ncw) <= 2 * rb;
}

void chain_prepare(int lds_bytes) {
  set_lds_limit<1, 1>(lds_bytes);
  set_lds_limit<1, 2>(lds_bytes);
  set_lds_limit<2, 1>(lds_bytes);
  set_lds_limit<2, 2>(lds_bytes);
  set_lds_limit<2, 3>(lds_bytes);
  set_lds_limit<2, 4>(lds_bytes);
  set_lds_limit<3, 1>(lds_bytes);
  set_lds_limit<3, 2>(lds_bytes);
  set_lds_limit<3, 3>(lds_bytes);
  set_lds_limit<3, 4>(lds_bytes);
  set_lds_limit<3, 5>(lds_bytes);
  set_lds_limit<3, 6>(lds_bytes);
}

void launch_chain_bwd(const ChainArgs& a, hipStream_t s) { launch_chain<true>(a, s); }
void launch_chain_fwd(const ChainArgs& a, hipStream_t s) { launch_chain<false>(a, s); }

}  // namespace cvb
