// Fused chains of dense layers (gfx950, FP32 MFMA).
//
// A workgroup owns T rows (subdomain x spec row) and carries them through a
// run of consecutive dense layers without leaving the chip: the current
// Lambda (back-substitution) or zhat (adjoint) of its rows lives in LDS and the
// weights stream from L2.
//
//   chain_bwd: top ReLU layer (relaxation of A(L-1) = C W(L), Sec. 2.1 /
//     Lemma 2.1) -> A(i-1) = Lambda(i) W(i) for i = L-1 .. lo (Eq.
//     definition_A), each followed by the next layer's relaxation; the last
//     step concretises over the box (Eq. beta_crown_lp) or writes the relaxed
//     Lambda(lo-1) to HBM for a convolution layer.
//   chain_fwd: zbar(i) = W(i) zhat(i-1) + b(i) for i = lo .. L-1, zhat(lo-1)
//     read from HBM, with the adjoint's gradients (or the fused Adam step).
//
// Each layer runs in two phases.  The MMA phase: 16x16x4 f32 MFMA blocks, a
// wave owning (16-column, 16-row) units round-robin, each lane feeding four
// consecutive k of one row (one b128 read) to four MFMAs; raw results go to
// LDS.  The relaxation phase: every thread takes one row and a strided set of
// columns and applies the per-neuron step with batched, independent loads
// (status record and chord, then alpha / beta), so the gathers of a whole
// tile are in flight together instead of one dependent chain per element.
#include "common.h"
#include "internal.h"

typedef float floatx4 __attribute__((ext_vector_type(4)));

namespace cvb {

namespace {

constexpr int G = 4;  // MMA units per register group
constexpr int E = 8;  // elements per thread per relaxation batch

template <int T>
__device__ __forceinline__ void init_rows(const Batch& bt, int r0, RowInfo* rinfo) {
  if (threadIdx.x < T) {
    const int row = r0 + threadIdx.x;
    if (row < bt.n_rows) rinfo[threadIdx.x] = row_info(bt, row);
  }
}

// Both LDS tiles start at zero: the k-chunk pairs read up to the next
// 32-multiple of a layer's width (finite values times zero-padded weights).
template <int T>
__device__ __forceinline__ void zero_tiles(float* sm, int ldk) {
  for (int t = threadIdx.x; t < 2 * T * ldk; t += 256) sm[t] = 0.f;
}

// acc[g] += A(rows of unit g) * Bt(cols of unit g)^T over K, A from LDS.
// The weight operand is zero-padded (rows to 16-multiples, K to 32-multiples)
// and the LDS tiles are zero-initialised, so k-chunks are processed in
// unconditional pairs on in-bounds data: the loads feed the MFMAs directly.
__device__ __forceinline__ void unit_mma(const ChainLayer& L, const float* cur, int ldk, const int* ucb,
                                         const int* urb, floatx4* acc) {
  const int lane = threadIdx.x & 63;
  const int KC = ((L.K + 31) >> 5) << 1;  // even number of 16-k chunks
  const int kq = 4 * (lane >> 4);
  const int nbm1 = ((L.N + 15) >> 4) - 1;
  const int kmax = KC * 16 - 4;
  const float* bp[G];
  const float* ap[G];
#pragma unroll
  for (int g = 0; g < G; ++g) {
    bp[g] = L.Bt + (int64_t)(min(ucb[g], nbm1) * 16 + (lane & 15)) * L.ldb;
    ap[g] = cur + (urb[g] * 16 + (lane & 15)) * ldk + kq;
  }
  auto ldb4 = [&](int g, int kc) {
    return *reinterpret_cast<const float4*>(bp[g] + min(kc * 16 + kq, kmax));
  };
  auto mma = [&](const float4* b, int kc) {
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const float4 af = *reinterpret_cast<const float4*>(ap[g] + kc * 16);
      acc[g] = __builtin_amdgcn_mfma_f32_16x16x4f32(af.x, b[g].x, acc[g], 0, 0, 0);
      acc[g] = __builtin_amdgcn_mfma_f32_16x16x4f32(af.y, b[g].y, acc[g], 0, 0, 0);
      acc[g] = __builtin_amdgcn_mfma_f32_16x16x4f32(af.z, b[g].z, acc[g], 0, 0, 0);
      acc[g] = __builtin_amdgcn_mfma_f32_16x16x4f32(af.w, b[g].w, acc[g], 0, 0, 0);
    }
  };
  float4 b0[G], b1[G];
#pragma unroll
  for (int g = 0; g < G; ++g) {
    b0[g] = ldb4(g, 0);
    b1[g] = ldb4(g, 1);
  }
  for (int kc = 0; kc < KC; kc += 2) {
    mma(b0, kc);
#pragma unroll
    for (int g = 0; g < G; ++g) b0[g] = ldb4(g, kc + 2);  // past the end: clamped, unused
    mma(b1, kc + 1);
#pragma unroll
    for (int g = 0; g < G; ++g) b1[g] = ldb4(g, kc + 3);
  }
}

// Raw products for output columns [col0, col0 + ncols) (ncols a 16-multiple)
// into dst[row][col - col0].
template <int T>
__device__ __forceinline__ void mma_phase(const ChainLayer& L, const float* cur, float* dst, int ldk, int col0,
                                          int ncols) {
  constexpr int RB = T / 16;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int rsub = 4 * (lane >> 4), csub = lane & 15;
  const int cb0 = col0 >> 4;
  const int nunits = (ncols >> 4) * RB;
  for (int u0 = wid; u0 < nunits; u0 += 4 * G) {
    int ucb[G], urb[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int u = min(u0 + 4 * g, nunits - 1);
      ucb[g] = cb0 + u / RB;
      urb[g] = u - (u / RB) * RB;
    }
    floatx4 acc[G];
#pragma unroll
    for (int g = 0; g < G; ++g) acc[g] = floatx4{0.f, 0.f, 0.f, 0.f};
    unit_mma(L, cur, ldk, ucb, urb, acc);
#pragma unroll
    for (int g = 0; g < G; ++g) {
      if (u0 + 4 * g >= nunits) continue;
      const int c = (ucb[g] - cb0) * 16 + csub;
#pragma unroll
      for (int r = 0; r < 4; ++r) dst[(urb[g] * 16 + rsub + r) * ldk + c] = acc[g][r];
    }
  }
}

// Relaxation of one row's neurons j = sub, sub + TPR, ... < n of the ReLU layer
// at nd-offset `off`: Lambda = relax(src), constants into *cst, result to dst.
// src / dst may alias (in place in LDS).
template <int TPR>
__device__ __forceinline__ void relax_phase(const ChainArgs& a, const RowInfo& ri, const float* src, float* dst,
                                            int n, int off, const float* bias, int sub, float* cst) {
  const uint32_t* st = a.bt.status + (int64_t)ri.b * a.bt.nd + off;
  const float2* chp = a.bt.chord + (int64_t)ri.p * a.bt.nd + off;
  for (int j0 = sub; j0 < n; j0 += TPR * E) {
    uint32_t rec[E];
    float2 ch[E];
    float av[E], bs[E], cf[E];
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
      cf[e] = relax_coef(a.bt, a.v, ri, rec[e], pc);
      if (a.v.acomp && (rec[e] & kKindMask) == kUnstable) a.v.acomp[ri.abase + (rec[e] & kCidxMask)] = av[e];
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int j = j0 + TPR * e;
      if (j < n) dst[j] = relax_value(a.bt, a.v, ri, rec[e], ch[e], cf[e], av[e], bs[e], cst);
    }
  }
}

// Box concretisation of one row's slab: columns col0 + 32 w + t for words
// w = sub, sub + TPR, ...; sign planes of A(0) stored a 32-bit word at a time.
template <int TPR>
__device__ __forceinline__ void conc_phase(const ChainArgs& a, const RowInfo& ri, int row, const float* src,
                                           int col0, int ncols, int n, int sub, float* cst) {
  const float* xl = a.bt.xlo + (int64_t)ri.p * a.bt.d0;
  const float* xu = a.bt.xhi + (int64_t)ri.p * a.bt.d0;
  const int nw = (ncols + 31) >> 5;
  for (int w = sub; w < nw; w += TPR) {
    uint32_t bp = 0, bn = 0;
#pragma unroll
    for (int q = 0; q < 32; q += 8) {
      float av[8], l8[8], u8[8];
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const int c = col0 + 32 * w + q + t;
        const bool ok = c < n;
        av[t] = src[32 * w + q + t];
        l8[t] = ok ? xl[c] : 0.f;
        u8[t] = ok ? xu[c] : 0.f;
      }
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const int c = col0 + 32 * w + q + t;
        if (c < n) {
          *cst += conc_term(av[t], l8[t], u8[t]);
          bp |= (av[t] > 0.f ? 1u : 0u) << (q + t);
          bn |= (av[t] < 0.f ? 1u : 0u) << (q + t);
        }
      }
    }
    if (a.v.xpos) {
      reinterpret_cast<uint32_t*>(a.v.xpos + (int64_t)row * a.bt.w64)[(col0 >> 5) + w] = bp;
      reinterpret_cast<uint32_t*>(a.v.xneg + (int64_t)row * a.bt.w64)[(col0 >> 5) + w] = bn;
    }
  }
}

template <int T>
__global__ __launch_bounds__(256) void chain_bwd(ChainArgs a) {
  constexpr int TPR = 256 / T;
  extern __shared__ __attribute__((aligned(16))) float sm[];
  __shared__ RowInfo rinfo[T];
  float* cur = sm;
  float* nxt = sm + T * a.ldk;
  const int tid = threadIdx.x;
  const int r0 = blockIdx.x * T;
  const int R = a.bt.n_rows;
  init_rows<T>(a.bt, r0, rinfo);
  zero_tiles<T>(sm, a.ldk);
  __syncthreads();
  const int rl = tid / TPR, sub = tid - rl * TPR;
  const int row = r0 + rl;
  const bool rok = row < R;
  RowInfo ri{};
  if (rok) ri = rinfo[rl];
  float cst = 0.f;

  // top ReLU layer: Lambda(L-1) = relax(C W(L)) into LDS
  if (rok)
    relax_phase<TPR>(a, ri, a.CW + ri.p * a.cw_pstride + (int64_t)ri.k * a.ldcw, cur + rl * a.ldk, a.n_top,
                     a.top_off, a.top_bias, sub, &cst);
  __syncthreads();

  const int nslab = a.ldk - 4;  // columns staged per slab of the last step (a 32-multiple)
  for (int s = 0; s < a.nl; ++s) {
    const ChainLayer L = a.ly[s];
    const int n16 = (L.N + 15) & ~15;
    if (s < a.nl - 1) {
      mma_phase<T>(L, cur, nxt, a.ldk, 0, n16);
      __syncthreads();
      if (rok) relax_phase<TPR>(a, ri, nxt + rl * a.ldk, nxt + rl * a.ldk, L.N, L.out_off, L.bias, sub, &cst);
      __syncthreads();
      float* t = cur;
      cur = nxt;
      nxt = t;
    } else {
      for (int c0 = 0; c0 < n16; c0 += nslab) {
        const int nc = min(nslab, n16 - c0);
        mma_phase<T>(L, cur, nxt, a.ldk, c0, nc);
        __syncthreads();
        if (rok) {
          if (a.conc)
            conc_phase<TPR>(a, ri, row, nxt + rl * a.ldk, c0, nc, L.N, sub, &cst);
          else
            relax_phase<TPR>(a, ri, nxt + rl * a.ldk, a.out + (int64_t)row * a.ldo + c0, min(nc, L.N - c0),
                             L.out_off + c0, L.bias + c0, sub, &cst);
        }
        __syncthreads();
      }
    }
  }

  // per-row constant: sum over the row's TPR lanes, plus the specification bias
#pragma unroll
  for (int o = TPR / 2; o > 0; o >>= 1) cst += __shfl_xor(cst, o, 64);
  if (sub == 0 && rok) {
    const float tot = cst + a.Cb[ri.p * a.cb_pstride + ri.k];
    if (a.final) {
      if (a.lb) a.lb[row] = tot;
      if (a.best) a.best[row] = a.first ? tot : fmaxf(a.best[row], tot);
    } else {
      a.part[(int64_t)a.slot * R + row] = tot;
    }
  }
}

// Adjoint step of one row's neurons j = sub, sub + TPR, ... < n of ReLU layer
// `off`: zhat = D (zbar + b) + lowerb written in place; gradients or Adam.
template <int TPR>
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

template <int T>
__global__ __launch_bounds__(256) void chain_fwd(ChainArgs a) {
  constexpr int TPR = 256 / T;
  extern __shared__ __attribute__((aligned(16))) float sm[];
  __shared__ RowInfo rinfo[T];
  float* cur = sm;
  float* nxt = sm + T * a.ldk;
  const int tid = threadIdx.x;
  const int r0 = blockIdx.x * T;
  const int R = a.bt.n_rows;
  init_rows<T>(a.bt, r0, rinfo);
  zero_tiles<T>(sm, a.ldk);
  __syncthreads();
  {
    // zhat(lo-1) of the tile's rows
    const int K = a.ly[0].K;
    for (int t = tid; t < T * K; t += 256) {
      const int r = t / K, k = t - r * K;
      if (r0 + r < R) cur[r * a.ldk + k] = a.in[(int64_t)(r0 + r) * a.ldi + k];
    }
  }
  __syncthreads();
  const int rl = tid / TPR, sub = tid - rl * TPR;
  const int row = r0 + rl;
  const bool rok = row < R;
  RowInfo ri{};
  if (rok) ri = rinfo[rl];
  for (int s = 0; s < a.nl; ++s) {
    const ChainLayer L = a.ly[s];
    const bool last = s == a.nl - 1;
    mma_phase<T>(L, cur, nxt, a.ldk, 0, (L.N + 15) & ~15);
    __syncthreads();
    if (rok) relax_fwd_phase<TPR>(a, ri, nxt + rl * a.ldk, L.N, L.out_off, L.bias, sub, !last);
    __syncthreads();
    float* t = cur;
    cur = nxt;
    nxt = t;
  }
}

}  // namespace

size_t chain_smem_bytes(int T, int ldk) { return (size_t)2 * T * ldk * sizeof(float); }

void launch_chain_bwd(int T, const ChainArgs& a, hipStream_t s) {
  const size_t sm = chain_smem_bytes(T, a.ldk);
  const unsigned grid = (unsigned)((a.bt.n_rows + T - 1) / T);
  if (T == 16) chain_bwd<16><<<grid, 256, sm, s>>>(a);
  else chain_bwd<32><<<grid, 256, sm, s>>>(a);
}

void launch_chain_fwd(int T, const ChainArgs& a, hipStream_t s) {
  const size_t sm = chain_smem_bytes(T, a.ldk);
  const unsigned grid = (unsigned)((a.bt.n_rows + T - 1) / T);
  if (T == 16) chain_fwd<16><<<grid, 256, sm, s>>>(a);
  else chain_fwd<32><<<grid, 256, sm, s>>>(a);
}

}  // namespace cvb
