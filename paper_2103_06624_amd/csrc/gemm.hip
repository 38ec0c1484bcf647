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

// 4 consecutive elements [k, k+4) of row `row` of a K-contiguous matrix
// (leading dimension ld >= K rounded up to 4, 16-byte aligned rows).  The
// address is clamped into the matrix, so the load needs no per-lane branch;
// mask4 zeroes what lies outside [0, nrows) x [0, K).  The two are separate
// so that the mask (which needs the data) runs when the slab is parked in
// LDS, not right after the load is issued.
__device__ __forceinline__ float4 ld4(const float* __restrict__ P, int ld, int row, int nrows, int k, int K) {
  const int K4 = (K + 3) & ~3;
  return *reinterpret_cast<const float4*>(P + (int64_t)min(row, nrows - 1) * ld + min(k, K4 - 4));
}

__device__ __forceinline__ float4 mask4(float4 x, int row, int nrows, int k, int K) {
  const bool rok = row < nrows;
  x.x = rok && k < K ? x.x : 0.f;
  x.y = rok && k + 1 < K ? x.y : 0.f;
  x.z = rok && k + 2 < K ? x.z : 0.f;
  x.w = rok && k + 3 < K ? x.w : 0.f;
  return x;
}

// Epilogue operands of one tile, gathered before its K loop so that they land
// while the MFMAs run.  Element (i, r, j) of a lane is row
// m0 + wm*WM + 16i + 4(lane/16) + r, column n0 + wn*WN + 16j + lane%16.
template <int BM, int BN>
struct TileOps {
  static constexpr int FM = BM / 32, FN = BN / 32, NE = FM * 4 * FN;
  RowInfo eri[FM][4];
  uint32_t rec[NE];
  float2 ech[NE];
  float ecf[NE], east[NE], ebias[FN];
  float ebe[NE];   // relaxation: beta of a split neuron (ecf holds alpha)
  float esw[NE];   // relaxation, sound mode: the neuron's rounding-error weight
  float2 emo[NE];  // adjoint with Adam: the moments of an unstable neuron's alpha
};

// OCC > 0 asks the compiler for at least OCC waves per SIMD (registers capped
// accordingly): with OCC = 8 a 32x32 tiling of ~10^4 x 200 is resident in one
// round instead of two.  DEPTH = 2 keeps two slabs of global loads in flight
// (two register sets, loads issued two slabs before they are parked in LDS):
// a slab's MFMA work is far shorter than the load latency at these sizes.
// DEPTH >= 3 holds all of K in registers (K <= DEPTH * BK): one load latency
// per tile instead of one per slab.
// Modes: kBwdRelax, kBwdConc, kFwd (the adjoint's first layer reads x* as a
// dense operand), kFwdTop (kFwd plus the next top-layer relaxation).
template <int BM, int BN, int BK, int MODE, int OCC, int DEPTH>
__global__ __launch_bounds__(256, OCC) void gemm_nt(const float* __restrict__ A, int lda, const float* __restrict__ Bt,
                                               int ldb, int M, int N, int K, int last, Batch bt, Vars v, Epi e) {
  constexpr int LDK = BK + 4;  // padded LDS row: LDK/4 odd, conflict-free b128 reads
  constexpr int WM = BM / 2, WN = BN / 2;
  constexpr int FM = WM / 16, FN = WN / 16;
  constexpr int QK = BK / 4;  // float4 per row of a slab
  constexpr int A_LD = (BM * QK + 255) / 256;  // float4 loads per thread
  constexpr int B_LD = (BN * QK + 255) / 256;
  using Ops = TileOps<BM, BN>;
  __shared__ __attribute__((aligned(16))) float As[2][BM][LDK];
  __shared__ __attribute__((aligned(16))) float Bs[2][BN][LDK];
  __shared__ float red[2][BM];
  __shared__ float rede[2][BM];  // sound mode: the rounding-error partials

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wid = tid >> 6;
  const int wm = wid >> 1, wn = wid & 1;
  const int rsub = 4 * (lane >> 4);
  const int csub = lane & 15;

  // XCD-aware order: consecutive logical tiles (the column tiles of one row
  // tile) land on the same XCD, so they share its L2 copy of the row tile.
  const int tiles_n = (N + BN - 1) / BN;
  const int nblk = gridDim.x;
  int logical = blockIdx.x;
  if ((nblk & 7) == 0) logical = (blockIdx.x & 7) * (nblk >> 3) + (blockIdx.x >> 3);
  const int tm = logical / tiles_n, tn = logical - tm * tiles_n;
  const int m0 = tm * BM, n0 = tn * BN;

  struct Regs {
    float4 a[A_LD], b[B_LD];
  };
  auto gload = [&](Regs& r, int k0) {
#pragma unroll
    for (int t = 0; t < A_LD; ++t) {
      const int idx = min(tid + t * 256, BM * QK - 1);
      r.a[t] = ld4(A, lda, m0 + idx / QK, M, k0 + (idx % QK) * 4, K);
    }
#pragma unroll
    for (int t = 0; t < B_LD; ++t) {
      const int idx = min(tid + t * 256, BN * QK - 1);
      r.b[t] = ld4(Bt, ldb, n0 + idx / QK, N, k0 + (idx % QK) * 4, K);
    }
  };
  // threads past the slab repeat its last float4 (same value, same address)
  auto sstore = [&](const Regs& r, int buf, int k0) {
#pragma unroll
    for (int t = 0; t < A_LD; ++t) {
      const int idx = min(tid + t * 256, BM * QK - 1);
      *reinterpret_cast<float4*>(&As[buf][idx / QK][(idx % QK) * 4]) =
          mask4(r.a[t], m0 + idx / QK, M, k0 + (idx % QK) * 4, K);
    }
#pragma unroll
    for (int t = 0; t < B_LD; ++t) {
      const int idx = min(tid + t * 256, BN * QK - 1);
      *reinterpret_cast<float4*>(&Bs[buf][idx / QK][(idx % QK) * 4]) =
          mask4(r.b[t], n0 + idx / QK, N, k0 + (idx % QK) * 4, K);
    }
  };
  auto compute = [&](floatx4 (&acc)[FM][FN], int buf) {
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
  };

  // epilogue operands, first level: bias, row info and status records
  auto gather1 = [&](Ops& o) {
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      const int col = n0 + wn * WN + j * 16 + csub;
      o.ebias[j] = (MODE != kBwdConc && col < N) ? e.bias[col] : 0.f;
    }
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm * WM + i * 16 + rsub + r;
        o.eri[i][r] = row_info(bt, min(row, M - 1));
#pragma unroll
        for (int j = 0; j < FN; ++j) {
          const int col = n0 + wn * WN + j * 16 + csub;
          const int q = (i * 4 + r) * FN + j;
          o.rec[q] = kInactive;
          if (MODE != kBwdConc && row < M && col < N)
            o.rec[q] = bt.status[(int64_t)o.eri[i][r].b * bt.nd + e.layer_off + col];
        }
      }
  };
  // second level, which needs the status records: chord and alpha / beta,
  // the stored A for the adjoint, or the box for concretisation
  auto gather2 = [&](Ops& o) {
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int j = 0; j < FN; ++j) {
          const int row = m0 + wm * WM + i * 16 + rsub + r;
          const int col = n0 + wn * WN + j * 16 + csub;
          const int q = (i * 4 + r) * FN + j;
          const RowInfo& ri = o.eri[i][r];
          o.ech[q] = make_float2(0.f, 0.f);
          o.ecf[q] = 0.f;
          o.east[q] = 0.f;
          o.ebe[q] = 0.f;
          o.esw[q] = 0.f;
          o.emo[q] = make_float2(0.f, 0.f);
          if (row >= M || col >= N) continue;
          if (MODE == kBwdConc) {
            const int64_t pb = (int64_t)ri.p * bt.d0 + col;
            o.ech[q] = bt.l2x0 ? make_float2(bt.l2x0[pb], 0.f) : make_float2(bt.xlo[pb], bt.xhi[pb]);
            continue;
          }
          const int64_t pc = (int64_t)ri.p * bt.nd + e.layer_off + col;
          const bool uns = (o.rec[q] & kKindMask) == kUnstable;
          if (uns) o.ech[q] = bt.chord[pc];
          if (MODE == kBwdRelax) {
            relax_vars(bt, v, ri, o.rec[q], pc, &o.ecf[q], &o.ebe[q]);
            if (bt.sw) o.esw[q] = bt.sw[pc];
          } else if (uns && !v.sat) {
            const int64_t ai = ri.abase + (o.rec[q] & kCidxMask);
            o.east[q] = v.acomp[ai];
            o.ecf[q] = v.alpha ? v.alpha[ai] : bt.adef[pc];
            if (v.adam) o.emo[q] = make_float2(v.ma[ai], v.va[ai]);
          }
          // the fused top layer: ebe holds C_p W(L) at this neuron
          if (MODE == kFwdTop) o.ebe[q] = e.cw[ri.p * e.cw_pstride + (int64_t)ri.k * e.ldcw + col];
        }
  };

  // epilogue: lane holds rows 4*(lane/16)+r of each 16x16 block, column lane%16
  auto epilogue = [&](const Ops& o, floatx4 (&acc)[FM][FN]) {
    if (MODE == kBwdRelax || MODE == kBwdConc) {
      // second per-row sum: the rounding-error bound (sound mode) or, when
      // concretising over an l2 ball, the sum of A(0)^2; with both modes on,
      // the other array's slot gets 0 (the l2 concretisation's own rounding is
      // bounded at the final sum)
      float* const p2 = MODE == kBwdConc && bt.l2x0 ? e.psq : (e.perr ? e.perr : e.psq);
      float* const pz = e.perr && e.psq ? (p2 == e.perr ? e.psq : e.perr) : nullptr;
      float cst[FM][4], cer[FM][4];
#pragma unroll
      for (int i = 0; i < FM; ++i) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          cst[i][r] = 0.f;
          cer[i][r] = 0.f;
          const int row = m0 + wm * WM + i * 16 + rsub + r;
          const bool rok = row < M;
          const RowInfo& ri = o.eri[i][r];
#pragma unroll
          for (int j = 0; j < FN; ++j) {
            const int col = n0 + wn * WN + j * 16 + csub;
            const int q = (i * 4 + r) * FN + j;
            const float a = acc[i][j][r];
            const bool ok = rok && col < N;
            if (MODE == kBwdRelax) {
              if (ok) {
                if (v.acomp && (o.rec[q] & kKindMask) == kUnstable) v.acomp[ri.abase + (o.rec[q] & kCidxMask)] = a;
                const float lam = relax_value(bt, v, ri, o.rec[q], o.ech[q], relax_pick(o.rec[q], o.ecf[q], o.ebe[q]),
                                              a, o.ebias[j], &cst[i][r]);
                e.out[(int64_t)row * e.ldo + col] = lam;
                cer[i][r] = fmaf(fabsf(lam), o.esw[q], cer[i][r]);
              }
            } else if (bt.l2x0) {  // l_p ball: A(0) x0 here, - eps ||A(0)||_q in the final sum
              if (ok) {
                cst[i][r] = fmaf(a, o.ech[q].x, cst[i][r]);
                const float xd = lp_entry(a, bt.lpq, &cer[i][r]);
                if (v.xdense) v.xdense[(int64_t)row * v.ldx + col] = xd;  // x*'s direction for the adjoint
              }
            } else {
              if (ok) {
                const float tm = conc_term(a, o.ech[q].x, o.ech[q].y);
                cst[i][r] += tm;
                cer[i][r] = fmaf(bt.sg, fabsf(tm), cer[i][r]);
              }
              if (ok && v.xdense) v.xdense[(int64_t)row * v.ldx + col] = xstar(a > 0.f, a < 0.f, o.ech[q].x, o.ech[q].y);
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
          if (p2) cer[i][r] = wave_sum16(cer[i][r]);
        }
      }
      // combine the two column halves (wn = 0, 1) of each row, one slot per tile
      if (csub == 0) {
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            red[wn][wm * WM + i * 16 + rsub + r] = cst[i][r];
            if (p2) rede[wn][wm * WM + i * 16 + rsub + r] = cer[i][r];
          }
      }
      __syncthreads();
      for (int t = tid; t < BM; t += 256) {
        const int row = m0 + t;
        if (row < M) {
          e.part[(int64_t)(e.slot0 + tn) * M + row] = red[0][t] + red[1][t];
          if (p2) p2[(int64_t)(e.slot0 + tn) * M + row] = rede[0][t] + rede[1][t];
          if (pz) pz[(int64_t)(e.slot0 + tn) * M + row] = 0.f;
        }
      }
    } else if (MODE == kFwdTop) {
      // last adjoint layer inside the optimiser: Adam step, then the next
      // iteration's top-layer relaxation with the new variables
      float cst[FM][4];
#pragma unroll
      for (int i = 0; i < FM; ++i) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          cst[i][r] = 0.f;
          const int row = m0 + wm * WM + i * 16 + rsub + r;
          const bool rok = row < M;
          const RowInfo& ri = o.eri[i][r];
#pragma unroll
          for (int j = 0; j < FN; ++j) {
            const int col = n0 + wn * WN + j * 16 + csub;
            const int q = (i * 4 + r) * FN + j;
            if (rok && col < N) {
              const float zb = e.wx0 ? fmaf(-v.l2s[row], acc[i][j][r], e.wx0[(int64_t)ri.p * N + col])
                                     : acc[i][j][r] + o.ebias[j];
              const int64_t pc = (int64_t)ri.p * bt.nd + e.layer_off + col;
              float vn = 0.f;
              relax_fwd_value(bt, v, ri, o.rec[q], o.ech[q], o.east[q], o.ecf[q], pc, zb, true, o.emo[q], &vn);
              const float a = o.ebe[q];
              if (v.acomp && (o.rec[q] & kKindMask) == kUnstable) v.acomp[ri.abase + (o.rec[q] & kCidxMask)] = a;
              e.top_out[(int64_t)row * e.ldo + col] = relax_value(bt, v, ri, o.rec[q], o.ech[q], vn, a, o.ebias[j],
                                                                  &cst[i][r]);
            }
          }
          cst[i][r] = wave_sum16(cst[i][r]);
        }
      }
      if (csub == 0) {
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int r = 0; r < 4; ++r) red[wn][wm * WM + i * 16 + rsub + r] = cst[i][r];
      }
      __syncthreads();
      for (int t = tid; t < BM; t += 256) {
        const int row = m0 + t;
        if (row < M) {
          float c = red[0][t] + red[1][t];
          if (tn == 0) {
            const RowInfo ri = row_info(bt, row);
            c += e.cb[ri.p * e.cb_pstride + ri.k];
          }
          e.part[(int64_t)(e.slot0 + tn) * M + row] = c;
          if (e.psq) e.psq[(int64_t)(e.slot0 + tn) * M + row] = 0.f;  // l2 ball: no A(0) terms here
        }
      }
    } else {
#pragma unroll
      for (int i = 0; i < FM; ++i) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = m0 + wm * WM + i * 16 + rsub + r;
          if (row >= M) continue;
          const RowInfo& ri = o.eri[i][r];
#pragma unroll
          for (int j = 0; j < FN; ++j) {
            const int col = n0 + wn * WN + j * 16 + csub;
            if (col >= N) continue;
            const int q = (i * 4 + r) * FN + j;
            // l2 ball, first layer: W(1) x* + b(1) = (W(1) x0 + b(1)) - l2s (W(1) A(0))
            const float zb = e.wx0 ? fmaf(-v.l2s[row], acc[i][j][r], e.wx0[(int64_t)ri.p * N + col])
                                   : acc[i][j][r] + o.ebias[j];
            if (v.sat) {  // the network itself at x*: every layer's output is kept
              e.out[(int64_t)row * e.ldo + col] = true_relu(o.rec[q], zb, v.sat + row);
              continue;
            }
            const int64_t pc = (int64_t)ri.p * bt.nd + e.layer_off + col;
            const float zh = relax_fwd_value(bt, v, ri, o.rec[q], o.ech[q], o.east[q], o.ecf[q], pc, zb, true, o.emo[q]);
            if (!last) e.out[(int64_t)row * e.ldo + col] = zh;
          }
        }
      }
    }
  };

  const int nk = (K + BK - 1) / BK;
  constexpr int NF = DEPTH >= 3 ? DEPTH : 1;
  Ops ops;
  Regs r0, r1, rf[NF];
  floatx4 acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};

  gather1(ops);
  if (DEPTH >= 3) {
#pragma unroll
    for (int d = 0; d < NF; ++d) gload(rf[d], min(d, nk - 1) * BK);
  } else {
    gload(r0, 0);
    if (DEPTH == 2) gload(r1, min(1, nk - 1) * BK);
  }
  gather2(ops);
  if (DEPTH >= 3) {
    // slab d sits in LDS buffer d & 1; slab d + 1 waits in rf[d + 1]
    sstore(rf[0], 0, 0);
    __syncthreads();
#pragma unroll
    for (int d = 0; d < NF; ++d) {
      if (d >= nk) break;
      compute(acc, d & 1);
      if (d + 1 < NF && d + 1 < nk) sstore(rf[d + 1 < NF ? d + 1 : 0], (d + 1) & 1, (d + 1) * BK);
      __syncthreads();
    }
  } else if (DEPTH == 1) {
    sstore(r0, 0, 0);
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
      const int buf = kt & 1;
      if (kt + 1 < nk) gload(r0, (kt + 1) * BK);
      compute(acc, buf);
      if (kt + 1 < nk) sstore(r0, buf ^ 1, (kt + 1) * BK);
      __syncthreads();
    }
  } else {
    // entering a pair of slabs kt, kt+1: slab kt in LDS buffer 0, slab kt+1
    // in flight in r1.  Loads and stores are unconditional (slab index
    // clamped: past the end they repeat the last slab into a buffer nobody
    // reads again), so every load is consumed on every path and no load is
    // left pending where its registers are reused.
    sstore(r0, 0, 0);
    __syncthreads();
    for (int kt = 0; kt < nk; kt += 2) {
      const int k2 = min(kt + 2, nk - 1) * BK, k3 = min(kt + 3, nk - 1) * BK;
      gload(r0, k2);
      compute(acc, 0);
      sstore(r1, 1, min(kt + 1, nk - 1) * BK);
      __syncthreads();
      if (kt + 1 >= nk) break;
      gload(r1, k3);
      compute(acc, 1);
      sstore(r0, 0, k2);
      __syncthreads();
    }
  }
  epilogue(ops, acc);
}

template <int BM, int BN, int BK, int OCC, int DEPTH>
void launch_cfg(int mode, const GemmArgs& g, hipStream_t s) {
  const int tiles = ((g.M + BM - 1) / BM) * ((g.N + BN - 1) / BN);
  dim3 grid(tiles), block(256);
  switch (mode) {
    case kBwdRelax:
      launch_k(gemm_nt<BM, BN, BK, kBwdRelax, OCC, DEPTH>, grid, block, 0, s, g.A, g.lda, g.Bt, g.ldb, g.M, g.N, g.K,
               g.last, g.bt, g.v, g.e);
      break;
    case kBwdConc:
      launch_k(gemm_nt<BM, BN, BK, kBwdConc, OCC, DEPTH>, grid, block, 0, s, g.A, g.lda, g.Bt, g.ldb, g.M, g.N, g.K,
               g.last, g.bt, g.v, g.e);
      break;
    case kFwdTop:
      launch_k(gemm_nt<BM, BN, BK, kFwdTop, OCC, DEPTH>, grid, block, 0, s, g.A, g.lda, g.Bt, g.ldb, g.M, g.N, g.K,
               g.last, g.bt, g.v, g.e);
      break;
    default:
      launch_k(gemm_nt<BM, BN, BK, kFwd, OCC, DEPTH>, grid, block, 0, s, g.A, g.lda, g.Bt, g.ldb, g.M, g.N, g.K,
               g.last, g.bt, g.v, g.e);
      break;
  }
}

}  // namespace

const GemmCfg kGemmCfgs[kNumGemmCfgs] = {
    {64, 64, 16, 0, 1}, {64, 32, 16, 0, 1}, {32, 64, 16, 0, 1}, {128, 64, 16, 0, 1}, {128, 32, 16, 0, 1},
    {32, 32, 16, 0, 1}, {32, 32, 32, 0, 1}, {32, 32, 64, 0, 1}, {64, 32, 32, 0, 1},  {32, 64, 32, 0, 1},
    {64, 64, 32, 0, 1}, {64, 32, 64, 0, 1}, {32, 64, 64, 0, 1}, {32, 32, 16, 8, 1},  {32, 32, 32, 8, 1},
    {64, 32, 16, 6, 1}, {32, 64, 16, 6, 1}, {32, 32, 16, 8, 2}, {32, 32, 32, 8, 2},  {32, 32, 32, 0, 2},
    {64, 32, 32, 0, 2}, {32, 64, 32, 0, 2}, {64, 64, 32, 0, 2}, {64, 32, 16, 6, 2},  {32, 64, 16, 6, 2},
    {32, 32, 64, 0, 2}, {64, 32, 64, 0, 2}, {32, 64, 64, 0, 2}, {64, 64, 16, 0, 2}, {64, 32, 32, 0, 8},
    {32, 32, 32, 0, 8}, {32, 64, 32, 0, 8}, {64, 64, 32, 0, 8}, {64, 32, 64, 0, 4}, {32, 32, 64, 0, 4},
    {32, 64, 64, 0, 4}, {64, 32, 32, 4, 2}, {32, 64, 32, 4, 2}, {64, 32, 16, 4, 2}, {64, 32, 32, 4, 1}};

bool gemm_cfg_fits(int cfg, int K) {
  const GemmCfg& c = kGemmCfgs[cfg];
  return c.depth <= 2 || (K + c.bk - 1) / c.bk <= c.depth;
}

void launch_gemm(int cfg, int mode, const GemmArgs& g, hipStream_t s) {
  if (!gemm_cfg_fits(cfg, g.K)) cfg = 19;  // K too deep for an all-of-K tiling
  switch (cfg) {
    case 0: launch_cfg<64, 64, 16, 0, 1>(mode, g, s); break;
    case 1: launch_cfg<64, 32, 16, 0, 1>(mode, g, s); break;
    case 2: launch_cfg<32, 64, 16, 0, 1>(mode, g, s); break;
    case 3: launch_cfg<128, 64, 16, 0, 1>(mode, g, s); break;
    case 4: launch_cfg<128, 32, 16, 0, 1>(mode, g, s); break;
    case 5: launch_cfg<32, 32, 16, 0, 1>(mode, g, s); break;
    case 6: launch_cfg<32, 32, 32, 0, 1>(mode, g, s); break;
    case 7: launch_cfg<32, 32, 64, 0, 1>(mode, g, s); break;
    case 8: launch_cfg<64, 32, 32, 0, 1>(mode, g, s); break;
    case 9: launch_cfg<32, 64, 32, 0, 1>(mode, g, s); break;
    case 10: launch_cfg<64, 64, 32, 0, 1>(mode, g, s); break;
    case 11: launch_cfg<64, 32, 64, 0, 1>(mode, g, s); break;
    case 12: launch_cfg<32, 64, 64, 0, 1>(mode, g, s); break;
    case 13: launch_cfg<32, 32, 16, 8, 1>(mode, g, s); break;
    case 14: launch_cfg<32, 32, 32, 8, 1>(mode, g, s); break;
    case 15: launch_cfg<64, 32, 16, 6, 1>(mode, g, s); break;
    case 16: launch_cfg<32, 64, 16, 6, 1>(mode, g, s); break;
    case 17: launch_cfg<32, 32, 16, 8, 2>(mode, g, s); break;
    case 18: launch_cfg<32, 32, 32, 8, 2>(mode, g, s); break;
    case 19: launch_cfg<32, 32, 32, 0, 2>(mode, g, s); break;
    case 20: launch_cfg<64, 32, 32, 0, 2>(mode, g, s); break;
    case 21: launch_cfg<32, 64, 32, 0, 2>(mode, g, s); break;
    case 22: launch_cfg<64, 64, 32, 0, 2>(mode, g, s); break;
    case 23: launch_cfg<64, 32, 16, 6, 2>(mode, g, s); break;
    case 24: launch_cfg<32, 64, 16, 6, 2>(mode, g, s); break;
    case 25: launch_cfg<32, 32, 64, 0, 2>(mode, g, s); break;
    case 26: launch_cfg<64, 32, 64, 0, 2>(mode, g, s); break;
    case 27: launch_cfg<32, 64, 64, 0, 2>(mode, g, s); break;
    case 28: launch_cfg<64, 64, 16, 0, 2>(mode, g, s); break;
    case 29: launch_cfg<64, 32, 32, 0, 8>(mode, g, s); break;
    case 30: launch_cfg<32, 32, 32, 0, 8>(mode, g, s); break;
    case 31: launch_cfg<32, 64, 32, 0, 8>(mode, g, s); break;
    case 32: launch_cfg<64, 64, 32, 0, 8>(mode, g, s); break;
    case 33: launch_cfg<64, 32, 64, 0, 4>(mode, g, s); break;
    case 34: launch_cfg<32, 32, 64, 0, 4>(mode, g, s); break;
    case 35: launch_cfg<32, 64, 64, 0, 4>(mode, g, s); break;
    case 36: launch_cfg<64, 32, 32, 4, 2>(mode, g, s); break;
    case 37: launch_cfg<32, 64, 32, 4, 2>(mode, g, s); break;
    case 38: launch_cfg<64, 32, 16, 4, 2>(mode, g, s); break;
    default: launch_cfg<64, 32, 32, 4, 1>(mode, g, s); break;
  }
}

}  // namespace cvb
