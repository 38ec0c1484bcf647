// Back-substitution and adjoint GEMMs for dense layers on FP32 MFMA (gfx950).
//
// Both directions are computed as C[M,N] = A[M,K] * Bt[N,K]^T with both
// operands K-contiguous:
//   back-substitution  A(i-1) = Lambda(i) W(i):  A = Lambda [rows, d_i],
//                      Bt = W(i)^T stored [d_{i-1}, d_i];
//   adjoint forward    zbar(i) = zhat(i-1) W(i)^T + b(i):  A = zhat,
//                      Bt = W(i) itself [d_i, d_{i-1}].
// The epilogue applies the next step of the method to the tile in registers:
// the ReLU relaxation of the next layer (Lemma 2.1 + beta S), the box
// concretisation (Eq. beta_crown_lp), or the adjoint's relaxed forward step
// with the alpha/beta gradients.
#include "common.h"
#include "internal.h"

typedef float floatx4 __attribute__((ext_vector_type(4)));

namespace cvb {

namespace {

template <int MODE>
__device__ __forceinline__ float4 load_a4(const float* __restrict__ A, int lda, int row, int k, int M, int K,
                                          const Batch& bt, const Vars& v) {
  float4 r = make_float4(0.f, 0.f, 0.f, 0.f);
  if (row >= M || k >= K) return r;
  if (MODE == kFwdX) {
    // zhat(0) = x*, rebuilt from the sign planes of A(0) and the box
    const int p = bt.prop[row / bt.m];
    const uint64_t wp = v.xpos[(int64_t)row * bt.w64 + (k >> 6)] >> (k & 63);
    const uint64_t wn = v.xneg[(int64_t)row * bt.w64 + (k >> 6)] >> (k & 63);
    const float* xl = bt.xlo + (int64_t)p * bt.d0 + k;
    const float* xu = bt.xhi + (int64_t)p * bt.d0 + k;
    if (k + 3 < K && (bt.d0 & 3) == 0) {
      const float4 l4 = *reinterpret_cast<const float4*>(xl);
      const float4 u4 = *reinterpret_cast<const float4*>(xu);
      r.x = xstar(wp & 1, wn & 1, l4.x, u4.x);
      r.y = xstar((wp >> 1) & 1, (wn >> 1) & 1, l4.y, u4.y);
      r.z = xstar((wp >> 2) & 1, (wn >> 2) & 1, l4.z, u4.z);
      r.w = xstar((wp >> 3) & 1, (wn >> 3) & 1, l4.w, u4.w);
      return r;
    }
    float t[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) t[q] = k + q < K ? xstar((wp >> q) & 1, (wn >> q) & 1, xl[q], xu[q]) : 0.f;
    return make_float4(t[0], t[1], t[2], t[3]);
  }
  const float* src = A + (int64_t)row * lda + k;
  if (k + 3 < K) return *reinterpret_cast<const float4*>(src);
  r.x = src[0];
  if (k + 1 < K) r.y = src[1];
  if (k + 2 < K) r.z = src[2];
  return r;
}

__device__ __forceinline__ float4 load_b4(const float* __restrict__ Bt, int ldb, int n, int k, int N, int K) {
  float4 r = make_float4(0.f, 0.f, 0.f, 0.f);
  if (n >= N || k >= K) return r;
  const float* src = Bt + (int64_t)n * ldb + k;
  if (k + 3 < K) return *reinterpret_cast<const float4*>(src);
  r.x = src[0];
  if (k + 1 < K) r.y = src[1];
  if (k + 2 < K) r.z = src[2];
  return r;
}

// 256 threads = 4 waves in a 2x2 arrangement; each wave owns (BM/2)x(BN/2)
// made of 16x16 MFMA blocks.  K advances BK at a time through double-buffered
// LDS tiles (the next slab's global loads are in flight while this one's
// MFMAs run, so a larger BK covers more latency); each lane reads 4
// consecutive k of one row with one b128 read and feeds them to 4 MFMAs (k
// slot g of MFMA t holds k = 4g + t, identically for both operands, so the
// products pair up correctly).
// OCC > 0 asks the compiler for at least OCC waves per SIMD (registers capped
// accordingly): with OCC = 8 a 32x32 tiling of ~10^4 x 200 is resident in one
// round instead of two.
template <int BM, int BN, int BK, int MODE, int OCC>
__global__ __launch_bounds__(256, OCC) void gemm_nt(const float* __restrict__ A, int lda, const float* __restrict__ Bt,
                                               int ldb, int M, int N, int K, int last, Batch bt, Vars v, Epi e) {
  constexpr int LDK = BK + 4;  // padded LDS row: LDK/4 odd, conflict-free b128 reads
  constexpr int WM = BM / 2, WN = BN / 2;
  constexpr int FM = WM / 16, FN = WN / 16;
  constexpr int QK = BK / 4;  // float4 per row of a slab
  constexpr int A_LD = (BM * QK + 255) / 256;  // float4 loads per thread
  constexpr int B_LD = (BN * QK + 255) / 256;
  __shared__ __attribute__((aligned(16))) float As[2][BM][LDK];
  __shared__ __attribute__((aligned(16))) float Bs[2][BN][LDK];
  __shared__ float red[2][BM];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wid = tid >> 6;
  const int wm = wid >> 1, wn = wid & 1;

  // XCD-aware order: consecutive logical tiles (the column tiles of one row
  // tile) land on the same XCD, so they share its L2 copy of the row tile.
  const int tiles_n = (N + BN - 1) / BN;
  const int nblk = gridDim.x;
  int logical = blockIdx.x;
  if ((nblk & 7) == 0) logical = (blockIdx.x & 7) * (nblk >> 3) + (blockIdx.x >> 3);
  const int tm = logical / tiles_n, tn = logical - tm * tiles_n;
  const int m0 = tm * BM, n0 = tn * BN;

  floatx4 acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};

  float4 ra[A_LD], rb[B_LD];
  auto gload = [&](int k0) {
#pragma unroll
    for (int t = 0; t < A_LD; ++t) {
      const int idx = tid + t * 256;
      ra[t] = (idx < BM * QK) ? load_a4<MODE>(A, lda, m0 + idx / QK, k0 + (idx % QK) * 4, M, K, bt, v)
                              : make_float4(0.f, 0.f, 0.f, 0.f);
    }
#pragma unroll
    for (int t = 0; t < B_LD; ++t) {
      const int idx = tid + t * 256;
      rb[t] = (idx < BN * QK) ? load_b4(Bt, ldb, n0 + idx / QK, k0 + (idx % QK) * 4, N, K)
                              : make_float4(0.f, 0.f, 0.f, 0.f);
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int t = 0; t < A_LD; ++t) {
      const int idx = tid + t * 256;
      if (idx < BM * QK) *reinterpret_cast<float4*>(&As[buf][idx / QK][(idx % QK) * 4]) = ra[t];
    }
#pragma unroll
    for (int t = 0; t < B_LD; ++t) {
      const int idx = tid + t * 256;
      if (idx < BN * QK) *reinterpret_cast<float4*>(&Bs[buf][idx / QK][(idx % QK) * 4]) = rb[t];
    }
  };

  // ---- epilogue operands, gathered before the K loop so that they land
  // while the MFMAs run: row info and status records first, then what
  // depends on them (chord and alpha / beta, the stored A for the adjoint, or
  // the box for concretisation).  Element (i, r, j) of a lane is row
  // m0 + wm*WM + 16i + 4(lane/16) + r, column n0 + wn*WN + 16j + lane%16.
  constexpr int NE = FM * 4 * FN;
  const int rsub = 4 * (lane >> 4);
  const int csub = lane & 15;
  RowInfo eri[FM][4];
  uint32_t rec[NE];
  float2 ech[NE];
  float ecf[NE], east[NE], ebias[FN];
#pragma unroll
  for (int j = 0; j < FN; ++j) {
    const int col = n0 + wn * WN + j * 16 + csub;
    ebias[j] = (MODE != kBwdConc && col < N) ? e.bias[col] : 0.f;
  }
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = m0 + wm * WM + i * 16 + rsub + r;
      eri[i][r] = row_info(bt, min(row, M - 1));
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        const int col = n0 + wn * WN + j * 16 + csub;
        const int q = (i * 4 + r) * FN + j;
        rec[q] = kInactive;
        if (MODE != kBwdConc && row < M && col < N)
          rec[q] = bt.status[(int64_t)eri[i][r].b * bt.nd + e.layer_off + col];
      }
    }

  const int nk = (K + BK - 1) / BK;
  gload(0);

#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        const int row = m0 + wm * WM + i * 16 + rsub + r;
        const int col = n0 + wn * WN + j * 16 + csub;
        const int q = (i * 4 + r) * FN + j;
        const RowInfo& ri = eri[i][r];
        ech[q] = make_float2(0.f, 0.f);
        ecf[q] = 0.f;
        east[q] = 0.f;
        if (row >= M || col >= N) continue;
        if (MODE == kBwdConc) {
          const int64_t pb = (int64_t)ri.p * bt.d0 + col;
          ech[q] = make_float2(bt.xlo[pb], bt.xhi[pb]);
          continue;
        }
        const int64_t pc = (int64_t)ri.p * bt.nd + e.layer_off + col;
        const bool uns = (rec[q] & kKindMask) == kUnstable;
        if (uns) ech[q] = bt.chord[pc];
        if (MODE == kBwdRelax) {
          ecf[q] = relax_coef(bt, v, ri, rec[q], pc);
        } else if (uns) {
          const int64_t ai = ri.abase + (rec[q] & kCidxMask);
          east[q] = v.acomp[ai];
          ecf[q] = v.alpha ? v.alpha[ai] : bt.adef[pc];
        }
      }

  sstore(0);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < nk) gload((kt + 1) * BK);
#pragma unroll
    for (int ks = 0; ks < BK; ks += 16) {
      float4 fa[FM], fb[FN];
#pragma unroll
      for (int i = 0; i < FM; ++i)
        fa[i] = *reinterpret_cast<const float4*>(&As[buf][wm * WM + i * 16 + (lane & 15)][ks + 4 * (lane >> 4)]);
#pragma unroll
      for (int j = 0; j < FN; ++j)
        fb[j] = *reinterpret_cast<const float4*>(&Bs[buf][wn * WN + j * 16 + (lane & 15)][ks + 4 * (lane >> 4)]);
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) {
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[i].x, fb[j].x, acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[i].y, fb[j].y, acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[i].z, fb[j].z, acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[i].w, fb[j].w, acc[i][j], 0, 0, 0);
        }
    }
    if (kt + 1 < nk) sstore(buf ^ 1);
    __syncthreads();
  }

  // ---- epilogue: lane holds rows 4*(lane/16)+r of each 16x16 block, column lane%16
  if (MODE == kBwdRelax || MODE == kBwdConc) {
    float cst[FM][4];
#pragma unroll
    for (int i = 0; i < FM; ++i) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        cst[i][r] = 0.f;
        const int row = m0 + wm * WM + i * 16 + rsub + r;
        const bool rok = row < M;
        const RowInfo& ri = eri[i][r];
#pragma unroll
        for (int j = 0; j < FN; ++j) {
          const int col = n0 + wn * WN + j * 16 + csub;
          const int q = (i * 4 + r) * FN + j;
          const float a = acc[i][j][r];
          const bool ok = rok && col < N;
          if (MODE == kBwdRelax) {
            if (ok) {
              if (v.acomp && (rec[q] & kKindMask) == kUnstable) v.acomp[ri.abase + (rec[q] & kCidxMask)] = a;
              e.out[(int64_t)row * e.ldo + col] = relax_value(bt, v, ri, rec[q], ech[q], ecf[q], a, ebias[j], &cst[i][r]);
            }
          } else {
            if (ok) cst[i][r] += conc_term(a, ech[q].x, ech[q].y);
            if (ok && v.xdense) v.xdense[(int64_t)row * v.ldx + col] = xstar(a > 0.f, a < 0.f, ech[q].x, ech[q].y);
            if (v.xpos) {
              const uint64_t mp = __ballot(ok && a > 0.f);
              const uint64_t mn = __ballot(ok && a < 0.f);
              const int cb = n0 + wn * WN + j * 16;
              if (csub == 0 && rok && cb < N) {
                const int g = lane >> 4;
                reinterpret_cast<uint16_t*>(v.xpos + (int64_t)row * bt.w64)[cb >> 4] = (uint16_t)(mp >> (16 * g));
                reinterpret_cast<uint16_t*>(v.xneg + (int64_t)row * bt.w64)[cb >> 4] = (uint16_t)(mn >> (16 * g));
              }
            }
          }
        }
        cst[i][r] = wave_sum16(cst[i][r]);
      }
    }
    // combine the two column halves (wn = 0, 1) of each row, one slot per tile
    if (csub == 0) {
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) red[wn][wm * WM + i * 16 + rsub + r] = cst[i][r];
    }
    __syncthreads();
    for (int t = tid; t < BM; t += 256) {
      const int row = m0 + t;
      if (row < M) e.part[(int64_t)(e.slot0 + tn) * M + row] = red[0][t] + red[1][t];
    }
  } else {
#pragma unroll
    for (int i = 0; i < FM; ++i) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm * WM + i * 16 + rsub + r;
        if (row >= M) continue;
        const RowInfo& ri = eri[i][r];
#pragma unroll
        for (int j = 0; j < FN; ++j) {
          const int col = n0 + wn * WN + j * 16 + csub;
          if (col >= N) continue;
          const int q = (i * 4 + r) * FN + j;
          const float zb = acc[i][j][r] + ebias[j];
          const int64_t pc = (int64_t)ri.p * bt.nd + e.layer_off + col;
          const float zh = relax_fwd_value(bt, v, ri, rec[q], ech[q], east[q], ecf[q], pc, zb);
          if (!last) e.out[(int64_t)row * e.ldo + col] = zh;
        }
      }
    }
  }
}

template <int BM, int BN, int BK, int OCC>
void launch_cfg(int mode, const GemmArgs& g, hipStream_t s) {
  const int tiles = ((g.M + BM - 1) / BM) * ((g.N + BN - 1) / BN);
  dim3 grid(tiles), block(256);
  switch (mode) {
    case kBwdRelax:
      gemm_nt<BM, BN, BK, kBwdRelax, OCC><<<grid, block, 0, s>>>(g.A, g.lda, g.Bt, g.ldb, g.M, g.N, g.K, g.last, g.bt,
                                                                 g.v, g.e);
      break;
    case kBwdConc:
      gemm_nt<BM, BN, BK, kBwdConc, OCC><<<grid, block, 0, s>>>(g.A, g.lda, g.Bt, g.ldb, g.M, g.N, g.K, g.last, g.bt,
                                                                g.v, g.e);
      break;
    case kFwdX:
      gemm_nt<BM, BN, BK, kFwdX, OCC><<<grid, block, 0, s>>>(g.A, g.lda, g.Bt, g.ldb, g.M, g.N, g.K, g.last, g.bt, g.v,
                                                             g.e);
      break;
    default:
      gemm_nt<BM, BN, BK, kFwd, OCC><<<grid, block, 0, s>>>(g.A, g.lda, g.Bt, g.ldb, g.M, g.N, g.K, g.last, g.bt, g.v,
                                                            g.e);
      break;
  }
}

}  // namespace

const GemmCfg kGemmCfgs[kNumGemmCfgs] = {
    {64, 64, 16, 0}, {64, 32, 16, 0}, {32, 64, 16, 0}, {128, 64, 16, 0}, {128, 32, 16, 0}, {32, 32, 16, 0},
    {32, 32, 32, 0}, {32, 32, 64, 0}, {64, 32, 32, 0}, {32, 64, 32, 0},  {64, 64, 32, 0},  {64, 32, 64, 0},
    {32, 64, 64, 0}, {32, 32, 16, 8}, {32, 32, 32, 8}, {64, 32, 16, 6}, {32, 64, 16, 6}};

void launch_gemm(int cfg, int mode, const GemmArgs& g, hipStream_t s) {
  switch (cfg) {
    case 0: launch_cfg<64, 64, 16, 0>(mode, g, s); break;
    case 1: launch_cfg<64, 32, 16, 0>(mode, g, s); break;
    case 2: launch_cfg<32, 64, 16, 0>(mode, g, s); break;
    case 3: launch_cfg<128, 64, 16, 0>(mode, g, s); break;
    case 4: launch_cfg<128, 32, 16, 0>(mode, g, s); break;
    case 5: launch_cfg<32, 32, 16, 0>(mode, g, s); break;
    case 6: launch_cfg<32, 32, 32, 0>(mode, g, s); break;
    case 7: launch_cfg<32, 32, 64, 0>(mode, g, s); break;
    case 8: launch_cfg<64, 32, 32, 0>(mode, g, s); break;
    case 9: launch_cfg<32, 64, 32, 0>(mode, g, s); break;
    case 10: launch_cfg<64, 64, 32, 0>(mode, g, s); break;
    case 11: launch_cfg<64, 32, 64, 0>(mode, g, s); break;
    case 12: launch_cfg<32, 64, 64, 0>(mode, g, s); break;
    case 13: launch_cfg<32, 32, 16, 8>(mode, g, s); break;
    case 14: launch_cfg<32, 32, 32, 8>(mode, g, s); break;
    case 15: launch_cfg<64, 32, 16, 6>(mode, g, s); break;
    default: launch_cfg<32, 64, 16, 6>(mode, g, s); break;
  }
}

}  // namespace cvb
