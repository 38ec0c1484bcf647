// Back-substitution through convolution layers and the adjoint's forward
// convolution, as implicit GEMMs on the matrix cores (gfx950, FP32 MFMA
// 16x16x4).
//
// Each batch row is one GEMM D[m, n] = sum_k G[m, k] Wm[k, n] (ConvPlan):
//  * transposed convolution, A(i-1) = Lambda(i) W(i) (Theorem 3.1 through a
//    conv layer), in polyphase form.  With stride s, an output (y, x) =
//    (s yy + py, s xx + px) of stride-parity class (py, px) takes the taps
//    ky = ky0(py) + s a, kx = kx0(px) + s b, and the Lambda entries they
//    meet sit at (Y - a, X - b) with Y = yy + T(py), X = xx + T(px).  The
//    GEMM rows are indexed by (Y, X), so every class reads the same Lambda
//    window: the s^2 classes and the c_in channels share the N axis
//    (s^2 c_in columns), K runs over (c_out, a, b), and Wm[(co, a, b),
//    (py, px, ci)] = W[co, ci, ky0(py) + s a, kx0(px) + s b] (0 past the
//    kernel).
//  * forward convolution (the adjoint's step, and the network itself for
//    the upper bound): rows (oy, ox), K = (c_in, ky, kx) as im2col, N = c_out.
//  * with 8 or fewer columns, two horizontally adjacent outputs x = 2 X + px
//    share a GEMM row and the N axis holds (px, channel): K widens to the
//    k + s taps (k + 1 for a stride-1 transposed convolution) that the pair
//    reads, and no MFMA column is left empty.
// G is gathered from the row's input staged in LDS through per-row and
// per-column offset tables: each channel plane is staged inside a zero
// border as wide as the farthest tap, so a gather is one add and one LDS
// read and the zero padding is exact.  The results are scattered into an LDS copy of
// the output row (each output position has exactly one (m, n)), and the
// layer's epilogue (relaxation, concretisation, adjoint step) then walks the
// row in natural order with coalesced global traffic.  Workgroups are
// persistent over rows, so the weight matrix and tables are loaded into LDS
// once per workgroup.
#include "common.h"
#include "internal.h"

namespace cvb {

namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kPF = 4;  // per thread and row: input floats and output records loaded ahead
// s_waitcnt immediate for vmcnt(0) with the other counters left free (gfx9
// encoding: vmcnt bits 3:0 and 15:14, expcnt 6:4, lgkmcnt 11:8)
constexpr int kWaitVm0 = 0x0F70;
constexpr int kEU = 4;  // outputs per thread whose second-level operands are gathered together

// Sum of x over the block (256 threads), returned to thread 0.
__device__ __forceinline__ float block_sum(float x, float* red) {
  x = wave_sum(x);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = x;
  __syncthreads();
  return threadIdx.x == 0 ? (red[0] + red[1]) + (red[2] + red[3]) : 0.f;
}

// First-level epilogue operands of outputs j = j0 + tid + 256 u of a row:
// the status records (relaxation, adjoint), or the box / ball centre of the
// row's property (concretisation).  Independent of the GEMM, so they are
// loaded while it runs.
template <int MODE>
__device__ __forceinline__ void epi_first(const Batch& bt, const Epi& e, int row, int p, int j0, int dout,
                                          uint32_t (&rec)[kPF], float (&b1)[kPF], float (&b2)[kPF]) {
  const uint32_t* st = bt.status + (int64_t)(row / bt.m) * bt.nd + e.layer_off;
#pragma unroll
  for (int u = 0; u < kPF; ++u) {
    const int jc = min(j0 + (int)threadIdx.x + 256 * u, dout - 1);
    rec[u] = kInactive;
    b1[u] = b2[u] = 0.f;
    if (MODE == kBwdConc) {  // (b2 unused over an l2 ball)
      const int64_t pb = (int64_t)p * bt.d0 + jc;
      b1[u] = (bt.l2x0 ? bt.l2x0 : bt.xlo)[pb];
      b2[u] = bt.xhi[pb];
    } else {
      rec[u] = st[jc];
    }
  }
}

// Input floats t = t0 + tid + TB u of a row: the row of zin, or for a conv
// first layer's adjoint step (row property p) the box and the sign planes of
// A(0) (x* is formed when the row is staged).  The box is read through a row
// pointer uniform across the workgroup (p taken to a scalar register).  The
// N inputs of a lane need bit (lane % 32) of 2N 32-bit words of each plane
// per wave (inputs u: words (t0 + TB u) / 32 + 2 wave + {0, 1}): lane 2u + h
// loads word h of input u into g1 (plane A(0) > 0) and g2 (A(0) < 0), and
// the lanes fetch theirs from it when the row is staged (xstar_from).
template <int MODE, int N, int TB = 256>
__device__ __forceinline__ void in_load(const float* zin, int ldi, const Batch& bt, const Vars& v, int row, int p,
                                        int t0, int din, float (&s1)[N], float (&s2)[N], uint32_t& g1,
                                        uint32_t& g2) {
  static_assert(2 * N <= 64, "one word per lane");
  if constexpr (MODE == kFwdX) {
    const int pu = __builtin_amdgcn_readfirstlane(p);
    const float* const xl = bt.xlo + (int64_t)pu * bt.d0;
    const float* const xu = bt.xhi + (int64_t)pu * bt.d0;
#pragma unroll
    for (int u = 0; u < N; ++u) {
      const int tc = min(t0 + (int)threadIdx.x + TB * u, din - 1);
      s1[u] = xl[tc];
      s2[u] = xu[tc];
    }
    const int lane = (int)threadIdx.x & 63, l = min(lane, 2 * N - 1);
    const int wi = min(((t0 + TB * (l >> 1)) >> 5) + 2 * ((int)threadIdx.x >> 6) + (l & 1), 2 * bt.w64 - 1);
    g1 = reinterpret_cast<const uint32_t*>(v.xpos + (int64_t)row * bt.w64)[wi];
    g2 = reinterpret_cast<const uint32_t*>(v.xneg + (int64_t)row * bt.w64)[wi];
  } else {
#pragma unroll
    for (int u = 0; u < N; ++u) {
      const int tc = min(t0 + (int)threadIdx.x + TB * u, din - 1);
      s1[u] = zin[(int64_t)row * ldi + tc];
      s2[u] = 0.f;
    }
    g1 = g2 = 0;
  }
}

// x* at input u of the lane from the words in_load left in g1, g2 (every
// lane of the wave takes part: a cross-lane read)
__device__ __forceinline__ float xstar_from(int u, uint32_t g1, uint32_t g2, float xl, float xu) {
  const int lane = (int)threadIdx.x & 63, src = 2 * u + (lane >> 5);
  const uint32_t a = (uint32_t)__shfl((int)g1, src), b = (uint32_t)__shfl((int)g2, src);
  return xstar((a >> (lane & 31)) & 1, (b >> (lane & 31)) & 1, xl, xu);
}

// the property of a row, where the first layer's adjoint step stages x*
template <int MODE>
__device__ __forceinline__ int row_prop(const Batch& bt, int row) {
  return MODE == kFwdX ? bt.prop[row / bt.m] : 0;
}

// Staged slot of input float t: channel plane c = t / (gh gw) and position
// (y, x) inside it, shifted into the zero-bordered layout (exact division by
// multiply-high with ceil(2^32 / d), valid for t < 2^32 / d).
__device__ __forceinline__ int staged(const ConvPlan& pl, int t) {
  const int c = __umulhi((unsigned)t, pl.mgp);
  const int rem = t - c * (pl.gh * pl.gw);
  const int y = __umulhi((unsigned)rem, pl.mgw);
  return c * pl.pplane + pl.bofs + y * pl.gwp + (rem - y * pl.gw);
}

template <int MODE, int N, int TB = 256>
__device__ __forceinline__ void in_store(float* zi, const ConvPlan& pl, const Batch& bt, const Vars& v, int row,
                                         int t0, int din, const float (&s1)[N], const float (&s2)[N],
                                         uint32_t g1, uint32_t g2) {
  if (MODE == kFwdX) {
#pragma unroll
    for (int u = 0; u < N; ++u) {
      const int t = t0 + (int)threadIdx.x + TB * u;
      const float x = xstar_from(u, g1, g2, s1[u], s2[u]);
      if (t < din) zi[staged(pl, t)] = x;
    }
  } else {
#pragma unroll
    for (int u = 0; u < N; ++u) {
      const int t = t0 + (int)threadIdx.x + TB * u;
      if (t < din) zi[staged(pl, t)] = s1[u];
    }
  }
}

// The implicit GEMM of one batch row, D = G Wm, from the row staged in zi into
// its LDS output row zo: each wave takes 16-row tiles of m, all N tiles.
// With sct set, the output slot of every accumulator element comes from a
// table built once per workgroup (sct[(mtile NT + t) 64 + lane] holds the
// four slots of the lane; slots outside the plane point at a spare slot past
// the row), so the scatter is four unconditional LDS stores.  TR computes the
// transposed tile (the MFMA's operands swapped): a lane then holds one
// output position and four columns, and a store of the 16 lanes that share
// a column writes 16 neighbouring positions of one channel plane -- distinct
// LDS banks, where the 16 columns (channels a plane apart) of one position
// would all meet in one or two banks.
// One 16-row tile of m (row origin mex of the lane's row) over the K steps
// [ks_lo, ks_hi) (multiples of 4), accumulated into acc: four K steps per
// pass, their gathers and weight reads issued before the MFMAs that use them;
// weights from global memory are loaded one pass ahead.  A gather's offset is
// either the lane's row origin plus kuni[step] + kv (uni: no table read on
// its path; kuni read through the constant address space, so by scalar
// loads) or the table's entry.
template <int NT, bool WG, bool TR>
__device__ __forceinline__ void conv_gemm_tile(const ConvPlan& pl, const float* zi, const float* wl, int mex,
                                               const int4* kt, bool uni, int kv, int ks_lo, int ks_hi, int lane,
                                               floatx4 (&acc)[NT]) {
  typedef const int __attribute__((address_space(4)))* cint_ptr;
  const cint_ptr ku = (cint_ptr)pl.kuni;
  float bn[4][NT];
  if (WG) {
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int t = 0; t < NT; ++t) bn[q][t] = wl[((ks_lo + q) * NT + t) * 64];
  }
  auto pass = [&](int ks0, const float(&a)[4]) {
    float b[4][NT];
    if (WG) {
      const int kn = ks0 + 4 < ks_hi ? ks0 + 4 : ks0;  // the last pass reloads its own (unused)
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          b[q][t] = bn[q][t];
          bn[q][t] = wl[((kn + q) * NT + t) * 64];
        }
    } else {
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int t = 0; t < NT; ++t) b[q][t] = wl[((ks0 + q) * NT + t) * 64];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int t = 0; t < NT; ++t)
        acc[t] = TR ? __builtin_amdgcn_mfma_f32_16x16x4f32(b[q][t], a[q], acc[t], 0, 0, 0)
                    : __builtin_amdgcn_mfma_f32_16x16x4f32(a[q], b[q][t], acc[t], 0, 0, 0);
  };
  if (uni) {
    const float* const zr = zi + mex + kv;
    for (int ks0 = ks_lo; ks0 < ks_hi; ks0 += 4) {
      float a[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) a[q] = zr[ku[ks0 + q]];
      pass(ks0, a);
      if (!WG) {
        // every LDS read of the pass (four gathers, the weights) issued
        // before its four MFMAs: one LDS latency per pass, not one per MFMA
        __builtin_amdgcn_sched_group_barrier(0x100, 4 + 2 * NT, 0);
        __builtin_amdgcn_sched_group_barrier(0x008, 4 * NT, 0);
      }
    }
  } else {
    for (int ks0 = ks_lo; ks0 < ks_hi; ks0 += 4) {
      int4 ke[4];
      float a[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) ke[q] = kt[(ks0 + q) * 4 + (lane >> 4)];
#pragma unroll
      for (int q = 0; q < 4; ++q) a[q] = zi[mex + ke[q].x];
      pass(ks0, a);
    }
  }
}

// The lane's part kv of the split column offsets (ConvPlan::kuni), 0 without.
__device__ __forceinline__ int conv_kv(const ConvPlan& pl, const int4* kt, int lane) {
  typedef const int __attribute__((address_space(4)))* cint_ptr;
  return pl.kuni ? kt[lane >> 4].x - ((cint_ptr)pl.kuni)[0] : 0;
}

template <int NT, bool WG, int NW = 4, bool TR = false>
__device__ __forceinline__ void conv_gemm_row(const ConvPlan& pl, const float* zi, float* zo, const float* wl,
                                              const int4* mt, const int4* kt, const int4* ntb, int n_ks, int n_mt,
                                              int lane, int wave, const int4* sct = nullptr) {
  const bool uni = pl.kuni != nullptr;
  const int kv = conv_kv(pl, kt, lane);
  for (int mtile = wave; mtile < n_mt; mtile += NW) {
    const int4 me = mt[mtile * 16 + (lane & 15)];
    floatx4 acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = floatx4{0.f, 0.f, 0.f, 0.f};
    conv_gemm_tile<NT, WG, TR>(pl, zi, wl, me.x, kt, uni, kv, 0, n_ks, lane, acc);
    // lane holds rows 4 (lane / 16) + r of the tile, column lane % 16 (TR:
    // row lane % 16, columns 4 (lane / 16) + r)
    if (sct) {
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const int4 ad = sct[(mtile * NT + t) * 64 + lane];
        zo[ad.x] = acc[t][0];
        zo[ad.y] = acc[t][1];
        zo[ad.z] = acc[t][2];
        zo[ad.w] = acc[t][3];
      }
      continue;
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int4 ne = ntb[t * 16 + (lane & 15)];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int4 mo = mt[mtile * 16 + 4 * (lane >> 4) + r];
        const int y = pl.osy * mo.z + ne.x, x = pl.osx * mo.w + ne.y;
        if (ne.z >= 0 && (unsigned)y < (unsigned)pl.oh && (unsigned)x < (unsigned)pl.ow)
          zo[ne.z + y * pl.ow + x] = acc[t][r];
      }
    }
  }
}

// in_store with the staged slots of inputs t = tid + TB u precomputed (so)
template <int MODE, int N, int TB>
__device__ __forceinline__ void in_store_at(float* zi, const int (&so)[N], int din, const float (&s1)[N],
                                            const float (&s2)[N], uint32_t g1, uint32_t g2) {
#pragma unroll
  for (int u = 0; u < N; ++u) {
    const int t = (int)threadIdx.x + TB * u;
    const float x = MODE == kFwdX ? xstar_from(u, g1, g2, s1[u], s2[u]) : s1[u];
    if (t < din) zi[so[u]] = x;
  }
}

// Waves per SIMD asked of the compiler (register budget), as measured best:
// four for the first layer's forward step (five spills its prefetched sign
// words), five for the other forward steps with one N tile and four with
// several, the compiler's own choice for back-substitution with one.
template <int MODE, int NT>
constexpr int conv_occupancy() {
  return MODE == kFwdX ? 4 : MODE == kFwd ? (NT == 1 ? 5 : 4) : (NT >= 2 ? 4 : 1);
}

// WG: the weight matrix is read from global memory (L1/L2) instead of LDS,
// for matrices too large to leave room for more than two workgroups per CU
// (measured 25-29 % faster there, 5-8 % slower for small matrices).
template <int MODE, int NT, bool WG>
__global__ __launch_bounds__(256, (conv_occupancy<MODE, NT>())) void conv_mm(const float* __restrict__ zin, int ldi, ConvPlan pl, int M, int last,
                                               Batch bt, Vars v, Epi e) {
  extern __shared__ float4 smem4[];
  __shared__ float red[2][4];
  constexpr bool kBwd = MODE == kBwdRelax || MODE == kBwdConc;
  float* const wm = reinterpret_cast<float*>(smem4);
  const int nwm = WG ? 0 : pl.kpad * NT * 16;  // floats in LDS
  int4* const mt = reinterpret_cast<int4*>(wm + nwm);
  int4* const kt = mt + pl.mpad;
  int4* const ntb = kt + pl.kpad;
  float* const zi = reinterpret_cast<float*>(ntb + NT * 16);
  float* const zo = zi + ((pl.dinp + 3) & ~3);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

  for (int t = tid; t < nwm / 4; t += 256) smem4[t] = reinterpret_cast<const float4*>(pl.wm)[t];
  for (int t = tid; t < pl.mpad; t += 256) mt[t] = pl.mtab[t];
  for (int t = tid; t < pl.kpad; t += 256) kt[t] = pl.ktab[t];
  for (int t = tid; t < NT * 16; t += 256) ntb[t] = pl.ntab[t];
  for (int t = tid; t < pl.dinp; t += 256) zi[t] = 0.f;  // the borders stay zero: out-of-plane taps
  __syncthreads();  // before any thread stages a row over the zeroed planes

  // the first row's input; later rows' inputs are loaded during the previous
  // row's GEMM and stored after its epilogue
  float s1[kPF], s2[kPF];
  uint32_t g1, g2;
  // XCD-aware row order: workgroups are dealt round-robin over the 8 XCDs, so
  // the logical index (b mod 8) (G / 8) + b / 8 gives each XCD a contiguous
  // block of rows at every step, and the spec rows of one subdomain
  // (consecutive rows) share its status words in that XCD's L2
  int row = blockIdx.x;
  if ((gridDim.x & 7) == 0) row = (blockIdx.x & 7) * (gridDim.x >> 3) + (blockIdx.x >> 3);
  if (row < M)
    for (int t0 = 0; t0 < pl.din; t0 += 256 * kPF) {
      in_load<MODE>(zin, ldi, bt, v, row, row_prop<MODE>(bt, row), t0, pl.din, s1, s2, g1, g2);
      in_store<MODE>(zi, pl, bt, v, row, t0, pl.din, s1, s2, g1, g2);
    }
  __syncthreads();

  const int n_ks = pl.kpad >> 2, n_mt = pl.mpad >> 4;
  const float* const wl = (WG ? pl.wm : wm) + lane;
  for (; row < M; row += gridDim.x) {
    const int nrow = row + gridDim.x;
    const int p = bt.prop[row / bt.m];
    const int np = nrow < M ? row_prop<MODE>(bt, nrow) : 0;
    uint32_t rec[kPF];
    float b1[kPF], b2[kPF];
    epi_first<MODE>(bt, e, row, p, 0, pl.dout, rec, b1, b2);
    if (nrow < M) in_load<MODE>(zin, ldi, bt, v, nrow, np, 0, pl.din, s1, s2, g1, g2);

    // ---- the GEMM: one 16-row tile of m per wave at a time, all N tiles
    conv_gemm_row<NT, WG>(pl, zi, zo, wl, mt, kt, ntb, n_ks, n_mt, lane, wave);
    __syncthreads();

    // ---- epilogue over the output row in natural order: first-level
    // operands for 256 kPF outputs at a time (the first chunk's were loaded
    // ahead), then kEU outputs per thread of second-level gathers
    const RowInfo ri = row_info(bt, row);
    const int64_t pc0 = (int64_t)p * bt.nd + e.layer_off;
    float cst = 0.f, cer = 0.f;
    for (int j0 = 0; j0 < pl.dout; j0 += 256 * kPF) {
      // concretisation loads the next chunk's box one chunk ahead (measured
      // faster there; slower for the modes with second-level gathers)
      constexpr bool kAhead = MODE == kBwdConc;
      uint32_t rn[kPF];
      float bn1[kPF], bn2[kPF];
      const bool more = j0 + 256 * kPF < pl.dout;
      if (kAhead && more) epi_first<MODE>(bt, e, row, p, j0 + 256 * kPF, pl.dout, rn, bn1, bn2);
      if (!kAhead && j0 > 0) epi_first<MODE>(bt, e, row, p, j0, pl.dout, rec, b1, b2);
#pragma unroll
      for (int h = 0; h < kPF; h += kEU) {
        float a[kEU], al[kEU], be[kEU], sw[kEU], bias[kEU];
        float2 ch[kEU];
#pragma unroll
        for (int u = 0; u < kEU; ++u) {
          const int j = j0 + tid + 256 * (h + u);
          const int jc = min(j, pl.dout - 1);
          const uint32_t r = rec[h + u];
          a[u] = zo[jc];
          ch[u] = make_float2(0.f, 0.f);
          al[u] = be[u] = sw[u] = bias[u] = 0.f;
          if (MODE == kBwdConc) continue;
          // l2 ball, first layer: W(1) x* + b(1) = (W(1) x0 + b(1)) - l2s (W(1) A(0))
          bias[u] = !kBwd && e.wx0 ? e.wx0[(int64_t)p * e.n + jc] : e.bias[jc];
          if (!kBwd && v.sat) continue;
          if ((r & kKindMask) == kUnstable) ch[u] = bt.chord[pc0 + jc];
          if (MODE == kBwdRelax) {
            relax_vars(bt, v, ri, r, pc0 + jc, &al[u], &be[u]);
            if (bt.sw) sw[u] = bt.sw[pc0 + jc];
          } else if ((r & kKindMask) == kUnstable) {
            const int64_t ai = ri.abase + (r & kCidxMask);
            be[u] = v.acomp[ai];  // the stored A(i)_j
            al[u] = v.alpha ? v.alpha[ai] : bt.adef[pc0 + jc];
          }
        }
#pragma unroll
        for (int u = 0; u < kEU; ++u) {
          const int j = j0 + tid + 256 * (h + u);
          const bool ok = j < pl.dout;
          const uint32_t r = rec[h + u];
          if (MODE == kBwdRelax) {
            if (!ok) continue;
            if (v.acomp && (r & kKindMask) == kUnstable) v.acomp[ri.abase + (r & kCidxMask)] = a[u];
            const float lam = relax_value(bt, v, ri, r, ch[u], relax_pick(r, al[u], be[u]), a[u], bias[u], &cst);
            e.out[(int64_t)row * e.ldo + j] = lam;
            cer = fmaf(fabsf(lam), sw[u], cer);
          } else if (MODE == kBwdConc) {
            if (bt.l2x0) {  // l_p ball: A(0) x0 here, - eps ||A(0)||_q in the final sum
              if (!ok) continue;
              cst = fmaf(a[u], b1[h + u], cst);
              const float xd = lp_entry(a[u], bt.lpq, &cer);
              if (v.xdense) v.xdense[(int64_t)row * v.ldx + j] = xd;  // x*'s direction for the adjoint
              continue;
            }
            if (ok) {
              const float tm = conc_term(a[u], b1[h + u], b2[h + u]);
              cst += tm;
              cer = fmaf(bt.sg, fabsf(tm), cer);
            }
            if (v.xpos) {  // x* as sign planes: one 64-bit word per wave
              const uint64_t bp = __ballot(ok && a[u] > 0.f), bn = __ballot(ok && a[u] < 0.f);
              const int w0 = j0 + 256 * (h + u) + wave * 64;
              if (lane == 0 && w0 < pl.dout) {
                v.xpos[(int64_t)row * bt.w64 + (w0 >> 6)] = bp;
                v.xneg[(int64_t)row * bt.w64 + (w0 >> 6)] = bn;
              }
            }
          } else {
            if (!ok) continue;
            const float zb = e.wx0 ? fmaf(-v.l2s[row], a[u], bias[u]) : a[u] + bias[u];
            if (v.sat) {  // the network itself at x*: every layer's output is kept
              e.out[(int64_t)row * e.ldo + j] = true_relu(r, zb, v.sat + row);
              continue;
            }
            const float zh = relax_fwd_value(bt, v, ri, r, ch[u], be[u], al[u], pc0 + j, zb);
            if (!last) e.out[(int64_t)row * e.ldo + j] = zh;
          }
        }
      }
      if (kAhead && more) {
#pragma unroll
        for (int u = 0; u < kPF; ++u) {
          rec[u] = rn[u];
          b1[u] = bn1[u];
          b2[u] = bn2[u];
        }
      }
    }
    if (kBwd) {
      const float tot = block_sum(cst, red[0]);
      if (tid == 0) e.part[(int64_t)e.slot0 * M + row] = tot;
      // rounding-error bound, or the sum of A(0)^2 (l2 ball); with both modes
      // on, the other array's slot gets 0
      float* const p2 = MODE == kBwdConc && bt.l2x0 ? e.psq : (e.perr ? e.perr : e.psq);
      float* const pz = e.perr && e.psq ? (p2 == e.perr ? e.psq : e.perr) : nullptr;
      if (p2) {
        const float ter = block_sum(cer, red[1]);
        if (tid == 0) p2[(int64_t)e.slot0 * M + row] = ter;
      }
      if (pz && tid == 0) pz[(int64_t)e.slot0 * M + row] = 0.f;
    }
    // the next row's input (every wave is past this row's GEMM)
    if (nrow < M) {
      in_store<MODE>(zi, pl, bt, v, nrow, 0, pl.din, s1, s2, g1, g2);
      for (int t0 = 256 * kPF; t0 < pl.din; t0 += 256 * kPF) {
        in_load<MODE>(zin, ldi, bt, v, nrow, np, t0, pl.din, s1, s2, g1, g2);
        in_store<MODE>(zi, pl, bt, v, nrow, t0, pl.din, s1, s2, g1, g2);
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Subdomain-major variant.  A workgroup takes work units of up to `mu`
// consecutive specification rows of one subdomain (all m rows when m is
// small).  The rows of a unit share the subdomain's status records and its
// property's chords, biases and box, so those are loaded once per unit into
// registers (NJ outputs per thread: dout <= 512 NJ), and the layer's bias
// into LDS once per workgroup; each row's own variables (alpha or beta, the
// stored A and the Adam moments) are loaded one row ahead, and the next row's
// input (its first 512 NI floats; any rest after the epilogue) is loaded while
// the current row's GEMM runs.  The epilogue then finds its operands in
// registers and LDS: no dependent gather is left on a row's critical path.

constexpr int kSdThreads = 512;  // threads per workgroup of the subdomain-major kernel
constexpr int kSdWaves = kSdThreads / 64;

// Per-unit operands of outputs j = tid + 512 u: the status record and the
// chord; for concretisation the box (or the ball's centre) in ch.
template <int MODE, int NJ>
__device__ __forceinline__ void sd_load(const Batch& bt, const Epi& e, int b, int p, int dout, uint32_t (&rec)[NJ],
                                        float2 (&ch)[NJ]) {
#pragma unroll
  for (int u = 0; u < NJ; ++u) {
    const int jc = min((int)threadIdx.x + kSdThreads * u, dout - 1);
    rec[u] = kInactive;
    if (MODE == kBwdConc) {
      const int64_t pb = (int64_t)p * bt.d0 + jc;
      ch[u] = make_float2((bt.l2x0 ? bt.l2x0 : bt.xlo)[pb], bt.xhi[pb]);
    } else {
      rec[u] = bt.status[(int64_t)b * bt.nd + e.layer_off + jc];
      ch[u] = bt.chord[(int64_t)p * bt.nd + e.layer_off + jc];  // defined (zero) for stable neurons too
    }
  }
}

// An opaque copy (in the adjoint modes) of a value the subdomain-major
// kernels keep across a subdomain's rows: tests on it are then made where they
// are used, in the row loop, instead of being hoisted out of it as per-lane
// masks (a 64-bit scalar pair each, several per output unit, which spill).
// Measured: the adjoint kernels 2-4 % faster; the back-substitution ones 1-6 %
// slower (there the recomputed tests cost more than the spills), so they keep
// the hoisted form.
template <int MODE, class T>
__device__ __forceinline__ T per_row(T x) {
  if (MODE == kFwd || MODE == kFwdX) asm volatile("" : "+v"(x));
  return x;
}

// Back-substitution with relaxation, per output unit of a subdomain: the
// relaxation's case analysis (Lemma 2.1 with the split term) as numbers, so
// that the epilogue is straight arithmetic on them:
//   Lambda = a (ca + (a >= 0 ? ux x : su)) + sg x,  constant += min(a, 0) ci,
// with x the unit's variable (alpha of an unstable neuron, beta of a split
// one): active ca = 1; unstable ux = 1 and the chord's slope su and intercept
// ci; split z >= 0: ca = 1, sg = -1; split z < 0: sg = +1; every other
// coefficient 0.  Each case gives the operations, and the roundings, of the
// case analysis.  The variable of row k is vsrc[k vstr] (alpha: the row's
// block moves by the property's unstable count; beta: by one); a unit with
// no variable reads a finite dummy (its default slope), which every
// coefficient it meets is 0 for.  cix: the unstable index (the stored A's
// slot), else -1.
struct RelaxCoef {
  float ca, ux, sg, su, ci;
  int cix, vstr;
  const float* vsrc;
};

// (the records and chords of all units are loaded first, unconditionally --
// the chords are defined at every neuron -- so that they are in flight
// together: one memory round trip per unit of rows, not two per output)
template <int NJ>
__device__ __forceinline__ void sd_relax_coef(const Batch& bt, const Vars& v, const Epi& e, int b, int p, int dout,
                                              int64_t ab0, int uc, RelaxCoef (&cf)[NJ]) {
  uint32_t rr[NJ];
  float2 chv[NJ];
#pragma unroll
  for (int u = 0; u < NJ; ++u) {
    const int jc = min((int)threadIdx.x + kSdThreads * u, dout - 1);
    rr[u] = bt.status[(int64_t)b * bt.nd + e.layer_off + jc];
    chv[u] = bt.chord[(int64_t)p * bt.nd + e.layer_off + jc];
  }
#pragma unroll
  for (int u = 0; u < NJ; ++u) {
    const int jc = min((int)threadIdx.x + kSdThreads * u, dout - 1);
    const int64_t pc = (int64_t)p * bt.nd + e.layer_off + jc;
    const uint32_t r = rr[u];
    const uint32_t kind = r & kKindMask;
    const bool pos = (r & kSidePos) != 0;
    RelaxCoef c{0.f, 0.f, 0.f, 0.f, 0.f, -1, 0, bt.adef + pc};
    if (kind == kActive) c.ca = 1.f;
    if (kind == kUnstable) {
      c.ux = 1.f;
      c.su = chv[u].x;
      c.ci = chv[u].y;
      c.cix = (int)(r & kCidxMask);
      if (v.alpha) {
        c.vsrc = v.alpha + ab0 + c.cix;
        c.vstr = uc;
      }
    }
    if (kind == kSplit) {
      c.ca = pos ? 1.f : 0.f;
      c.sg = pos ? -1.f : 1.f;
      c.vsrc = v.beta + (int64_t)(r & kSplitMask) * bt.m;
      c.vstr = 1;
    }
    cf[u] = c;
  }
}

// Adjoint (the forward sweep from x*), per output unit of a subdomain: the
// relaxation's case analysis as numbers, like the back-substitution's.  With
// a the GEMM's output, zb = rm a + kb (kb the bias, or W(1) x0 + b(1) on an l2
// ball's first layer, where rm = -l2s of the row; rm = 1 otherwise), x1 the
// stored A(i)_j of an unstable neuron (0 elsewhere) and x2 its alpha
// (elsewhere the constant slope: 1 active or split z >= 0, 0 inactive or
// split z < 0):
//   zhat = x1 >= 0 ? zb x2 : su zb + ci,
// and an unstable neuron's alpha gradient is x1 >= 0 ? zb x1 : 0 -- the
// operations and roundings of the case analysis, the sign of a zero aside.
// cix: an unstable neuron's alpha slot; -2 - (its alpha slot) for a split
// neuron, whose record bits (side, split index) are bsp; -1 otherwise.  x1
// and x2 keep their constants over the unit's rows except at unstable
// neurons, whose A, alpha (and Adam moments x3, x4) each row loads.
struct AdjCoef {
  float su, ci;
  int cix;
  uint32_t bsp;
};

template <int NJ>
__device__ __forceinline__ void sd_adj_coef(const Batch& bt, const Vars& v, const Epi& e, int b, int p, int dout,
                                            AdjCoef (&cf)[NJ], float (&x1)[NJ], float (&x2)[NJ], float (&x3)[NJ],
                                            float (&x4)[NJ]) {
  // (all loads first, as for the back-substitution)
  uint32_t rr[NJ];
  float2 chv[NJ];
  float ad[NJ];
  int cx[NJ];
#pragma unroll
  for (int u = 0; u < NJ; ++u) {
    const int jc = min((int)threadIdx.x + kSdThreads * u, dout - 1);
    const int64_t pc = (int64_t)p * bt.nd + e.layer_off + jc;
    rr[u] = bt.status[(int64_t)b * bt.nd + e.layer_off + jc];
    chv[u] = bt.chord[pc];
    ad[u] = bt.adef[pc];
    cx[u] = bt.cidx[pc];
  }
#pragma unroll
  for (int u = 0; u < NJ; ++u) {
    const uint32_t r = rr[u];
    const uint32_t kind = (int)threadIdx.x + kSdThreads * u < dout ? r & kKindMask : kInactive;
    AdjCoef c{0.f, 0.f, -1, 0u};
    float ca = kind == kActive ? 1.f : 0.f;
    if (kind == kUnstable) {
      c.su = chv[u].x;
      c.ci = chv[u].y;
      c.cix = (int)(r & kCidxMask);
      ca = ad[u];  // the default alpha, for passes given none
    }
    if (kind == kSplit) {
      ca = (r & kSidePos) ? 1.f : 0.f;
      c.cix = -2 - cx[u];
      c.bsp = r & (kSidePos | kSplitMask);
    }
    cf[u] = c;
    x1[u] = 0.f;
    x2[u] = ca;
    x3[u] = x4[u] = 0.f;
  }
}

template <int MODE, int NJ>
__device__ __forceinline__ void sd_adj_row_vars(const Vars& v, const RowInfo& ri, const AdjCoef (&cf)[NJ],
                                                float (&x1)[NJ], float (&x2)[NJ], float (&x3)[NJ], float (&x4)[NJ]) {
  if (v.sat) return;
  const float* const ac = v.acomp + ri.abase;
#pragma unroll
  for (int u = 0; u < NJ; ++u) {
    const int ci = per_row<MODE>(cf[u].cix);
    if (ci >= 0) {
      // (unsigned offsets from the row's uniform base: scalar-base addressing)
      const uint32_t o = (uint32_t)ci;
      x1[u] = ac[o];
      if (v.alpha) x2[u] = (v.alpha + ri.abase)[o];
      if (v.adam) {
        x3[u] = (v.ma + ri.abase)[o];
        x4[u] = (v.va + ri.abase)[o];
      }
    }
  }
}

// A split neuron's variables (cix <= -2): beta's gradient is -zb on the
// z >= 0 side and zb on the z < 0 side; its alpha slot gets gradient 0 (with
// Adam: a step on its moments alone).
__device__ __forceinline__ void adj_split(const Batch& bt, const Vars& v, const RowInfo& ri, int cix, uint32_t bsp,
                                          float zb) {
  const int64_t bi = (int64_t)(bsp & kSplitMask) * bt.m + ri.k;
  const int64_t ai = ri.abase + (-2 - cix);
  const float gb = (bsp & kSidePos) ? -zb : zb;
  if (v.gsplit) {  // the steps: split_adam_k, after the pass
    v.gsplit[bi] = gb;
  } else if (v.adam) {
    adam_apply(v.beta_w, v.mb, v.vb, bi, gb, v.lr_b, v.bc1, v.bc2, 0.f, INFINITY);
    adam_apply(v.alpha_w, v.ma, v.va, ai, 0.f, v.lr_a, v.bc1, v.bc2, 0.f, 1.f);
  } else {
    v.gbeta[bi] = gb;
    v.galpha[ai] = 0.f;
  }
}

// The adjoint's epilogue of one row (the relaxed network; orow: the row of
// the next layer's input, or null after the last layer).
template <int MODE, bool kAdam, int NJ>
__device__ __forceinline__ void sd_adj_epi(const Batch& bt, const Vars& v, const RowInfo& ri, const float* zo,
                                           int dout, float rm, const float* kb, float* orow, const AdjCoef (&cf)[NJ],
                                           const float (&x1)[NJ], const float (&x2)[NJ], const float (&x3)[NJ],
                                           const float (&x4)[NJ]) {
#pragma unroll
  for (int u = 0; u < NJ; ++u) {
    const int j = per_row<MODE>((int)threadIdx.x + kSdThreads * u);
    if (j >= dout) continue;
    const AdjCoef& c = cf[u];
    const float zb = fmaf(rm, zo[j], kb[j]);
    const bool ge = x1[u] >= 0.f;
    const float zh = ge ? zb * x2[u] : fmaf(c.su, zb, c.ci);
    if (orow) orow[(uint32_t)j] = zh;
    const int ci = per_row<MODE>(c.cix);
    if (ci >= 0) {
      const float g = ge ? zb * x1[u] : 0.f;
      const uint32_t o = (uint32_t)ci;
      if (kAdam)
        adam_step(v.alpha_w + ri.abase, v.ma + ri.abase, v.va + ri.abase, o, g, v.lr_a, v.bc1, v.bc2, 0.f, 1.f,
                  x2[u], x3[u], x4[u]);
      else
        (v.galpha + ri.abase)[o] = g;
    } else if (ci < -1) {
      adj_split(bt, v, ri, ci, per_row<MODE>(c.bsp), zb);  // its addresses: computed here, not held
    }
  }
}

// The network itself at x* (upper bound): the exact ReLU, every layer's
// output kept; a pre-activation that breaks a split of the row's subdomain
// clears sat[row].
template <int MODE, int NJ>
__device__ __forceinline__ void sd_adj_sat(const Vars& v, const float* zo, int dout, float rm, const float* kb,
                                           float* orow, int row, const AdjCoef (&cf)[NJ]) {
#pragma unroll
  for (int u = 0; u < NJ; ++u) {
    const int j = per_row<MODE>((int)threadIdx.x + kSdThreads * u);
    if (j >= dout) continue;
    const AdjCoef& c = cf[u];
    const float zb = fmaf(rm, zo[j], kb[j]);
    if (c.cix < -1 && ((c.bsp & kSidePos) ? zb < 0.f : zb > 0.f)) v.sat[row] = 0;
    orow[j] = fmaxf(zb, 0.f);
  }
}

// The first layer's adjoint step in the subdomain-major kernel stages x* for
// the whole input row right after the GEMM: the lanes' words of the two sign
// planes for every 512-input chunk of the row (at most 32 chunks) come in one
// load per plane (lane 2u + h: word h of chunk u, as in_load), the box of the
// first NI chunks in registers, and that of the rest (the tail) from LDS, each
// thread holding the entries it stages itself (no barrier), rewritten when the
// next unit's first row is staged (the property may change there only).
__device__ __forceinline__ void sdx_words(const Batch& bt, const Vars& v, int row, uint32_t& g1, uint32_t& g2) {
  const int lane = (int)threadIdx.x & 63;
  const int wi = min(16 * (lane >> 1) + 2 * ((int)threadIdx.x >> 6) + (lane & 1), 2 * bt.w64 - 1);
  g1 = reinterpret_cast<const uint32_t*>(v.xpos + (int64_t)row * bt.w64)[wi];
  g2 = reinterpret_cast<const uint32_t*>(v.xneg + (int64_t)row * bt.w64)[wi];
}

template <int NI>
__device__ __forceinline__ void sdx_box(const Batch& bt, int p, int din, float (&s1)[NI], float (&s2)[NI]) {
  const int pu = __builtin_amdgcn_readfirstlane(p);
  const float* const xl = bt.xlo + (int64_t)pu * bt.d0;
  const float* const xu = bt.xhi + (int64_t)pu * bt.d0;
#pragma unroll
  for (int u = 0; u < NI; ++u) {
    const int tc = min((int)threadIdx.x + kSdThreads * u, din - 1);
    s1[u] = xl[tc];
    s2[u] = xu[tc];
  }
}

// the tail of property p's box into bxt ([2][din - kSdThreads NI]); din > kSdThreads NI
template <int NI>
__device__ __forceinline__ void sdx_tail_box(const Batch& bt, int p, int din, float* bxt) {
  const int base = kSdThreads * NI, nt = din - base;
  const int pu = __builtin_amdgcn_readfirstlane(p);
  const float* const xl = bt.xlo + (int64_t)pu * bt.d0 + base;
  const float* const xu = bt.xhi + (int64_t)pu * bt.d0 + base;
  for (int t = (int)threadIdx.x; t < nt; t += kSdThreads) {
    bxt[t] = xl[t];
    bxt[nt + t] = xu[t];
  }
}

template <int NI>
__device__ __forceinline__ void sdx_stage(float* zi, const ConvPlan& pl, int din, const float (&s1)[NI],
                                          const float (&s2)[NI], uint32_t g1, uint32_t g2, const float* bxt) {
#pragma unroll
  for (int u = 0; u < NI; ++u) {
    const int t = (int)threadIdx.x + kSdThreads * u;
    const float x = xstar_from(u, g1, g2, s1[u], s2[u]);
    if (t < din) zi[staged(pl, t)] = x;
  }
  const int base = kSdThreads * NI, nt = din - base;
  for (int u = NI; kSdThreads * u < din; ++u) {
    const int t = (int)threadIdx.x + kSdThreads * u, i = min(t - base, nt - 1);
    const float x = xstar_from(u, g1, g2, bxt[i], bxt[nt + i]);
    if (t < din) zi[staged(pl, t)] = x;
  }
}

// occupancy (waves per SIMD) of the subdomain-major kernels
template <int MODE, int NJ, int NI>
constexpr int conv_sd_occupancy() {
  // the adjoint holds four variables per output (stored A, alpha, Adam
  // moments) and the first layer's the sign-plane words of its input
  return NJ >= 8 || NJ + NI >= 12 ? 3 : 4;
}

template <int MODE, int NT, bool WG, int NJ, int NI>
__global__ __launch_bounds__(kSdThreads, (conv_sd_occupancy<MODE, NJ, NI>())) void conv_sd(
    const float* __restrict__ zin, int ldi, ConvPlan pl, int M, int last, Batch bt, Vars v, Epi e, int mu) {
  extern __shared__ float4 smem4[];
  __shared__ float red[2][kSdWaves][2];
  constexpr bool kBwd = MODE == kBwdRelax || MODE == kBwdConc;
  const int m = bt.m;
  const int upb = (m + mu - 1) / mu;  // units per subdomain
  const int n_units = (M / m) * upb;
  if ((int)blockIdx.x >= n_units) return;
  float* const wm = reinterpret_cast<float*>(smem4);
  const int nwm = WG ? 0 : pl.kpad * NT * 16;  // floats in LDS
  int4* const mt = reinterpret_cast<int4*>(wm + nwm);
  int4* const kt = mt + pl.mpad;
  int4* const ntb = kt + pl.kpad;
  float* const zi = reinterpret_cast<float*>(ntb + NT * 16);
  float* const zo = zi + ((pl.dinp + 3) & ~3);  // the output row, then a spare slot (padding: at most 7 floats)
  int4* const sct = reinterpret_cast<int4*>(zo + ((pl.dout + 4 + 3) & ~3));  // scatter slots [n_mt NT 64]
  const int n_mt = pl.mpad >> 4;
  float* const bsh = reinterpret_cast<float*>(sct + n_mt * NT * 64);  // bias per neuron (not for concretisation)
  // partial tiles of a split K (below): [kSdWaves][NT][64] floatx4
  floatx4* const kpart = reinterpret_cast<floatx4*>(bsh + (MODE != kBwdConc ? (pl.dout + 3) & ~3 : 0));
  // the first layer's adjoint step: the tail of the box (sdx_tail_box)
  float* const bxt = reinterpret_cast<float*>(kpart + (n_mt < kSdWaves && pl.kpad >= 32 ? kSdWaves * NT * 64 : 0));
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // With fewer 16-row tiles than waves (a small output plane with a long K),
  // each tile's K passes are split over ksp waves (a power of two, a pass at
  // least each) whose partial tiles are summed in LDS before the scatter.
  // (compiled in for the narrow output instantiations only, NJ <= 2: the
  // wide ones have planes of many tiles, and its registers would cost them)
  int ksp = 1;
  if (NJ <= 2)
    while (2 * ksp * n_mt <= kSdWaves && 2 * ksp <= (pl.kpad >> 4)) ksp *= 2;

  for (int t = tid; t < nwm / 4; t += kSdThreads) smem4[t] = reinterpret_cast<const float4*>(pl.wm)[t];
  for (int t = tid; t < pl.mpad; t += kSdThreads) mt[t] = pl.mtab[t];
  for (int t = tid; t < pl.kpad; t += kSdThreads) kt[t] = pl.ktab[t];
  for (int t = tid; t < NT * 16; t += kSdThreads) ntb[t] = pl.ntab[t];
  for (int t = tid; t < pl.dinp; t += kSdThreads) zi[t] = 0.f;  // the borders stay zero: out-of-plane taps
  if (MODE != kBwdConc)
    for (int t = tid; t < pl.dout; t += kSdThreads) bsh[t] = e.bias[t];
  __syncthreads();  // before any thread stages a row over the zeroed planes
  // the scatter slot of every accumulator element (the same for every row);
  // element r of lane l in tile (mtile, t) is output (m = 16 mtile + l % 16,
  // n = 16 t + 4 (l / 16) + r) (the transposed tile); outputs outside the
  // plane go to the spare slot
  for (int i = tid; i < n_mt * NT * 64; i += kSdThreads) {
    const int mtile = i / (NT * 64), t = (i / 64) % NT, ln = i % 64;
    const int4 mo = mt[mtile * 16 + (ln & 15)];
    int ad[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int4 ne = ntb[t * 16 + 4 * (ln >> 4) + r];
      const int y = pl.osy * mo.z + ne.x, x = pl.osx * mo.w + ne.y;
      const bool ok = ne.z >= 0 && (unsigned)y < (unsigned)pl.oh && (unsigned)x < (unsigned)pl.ow;
      ad[r] = ok ? ne.z + y * pl.ow + x : pl.dout;
    }
    sct[i] = make_int4(ad[0], ad[1], ad[2], ad[3]);
  }
  const bool uni = pl.kuni != nullptr;
  const int kv = conv_kv(pl, kt, lane);
  // the staged slots of this thread's first NI kSdThreads inputs (the same for every row)
  int so[NI];
#pragma unroll
  for (int u = 0; u < NI; ++u) so[u] = MODE == kFwdX ? 0 : staged(pl, min(tid + kSdThreads * u, pl.din - 1));

  // the first row of this workgroup's first unit: staged before the loop;
  // later units' first rows are staged by the previous row, like any next row
  {
    const int b0 = blockIdx.x / upb;
    const int row0 = b0 * m + ((int)blockIdx.x - b0 * upb) * mu;
    float s1[NI], s2[NI];
    uint32_t g1, g2;
    if constexpr (MODE == kFwdX) {
      const int p0 = bt.prop[b0];
      if (pl.din > kSdThreads * NI) sdx_tail_box<NI>(bt, p0, pl.din, bxt);
      sdx_box<NI>(bt, p0, pl.din, s1, s2);
      sdx_words(bt, v, row0, g1, g2);
      sdx_stage<NI>(zi, pl, pl.din, s1, s2, g1, g2, bxt);
    } else {
      for (int t0 = 0; t0 < pl.din; t0 += kSdThreads * NI) {
        in_load<MODE, NI, kSdThreads>(zin, ldi, bt, v, row0, 0, t0, pl.din, s1, s2, g1, g2);
        in_store<MODE, NI, kSdThreads>(zi, pl, bt, v, row0, t0, pl.din, s1, s2, g1, g2);
      }
    }
  }
  const int n_ks = pl.kpad >> 2;
  const float* const wl = (WG ? pl.wm : wm) + lane;
  int par = 0;
  for (int unit = blockIdx.x; unit < n_units; unit += gridDim.x) {
    const int b = unit / upb;
    const int r0 = b * m + (unit - b * upb) * mu;
    const int r1 = b * m + min((unit - b * upb) * mu + mu, m);
    const int p = bt.prop[b];
    // a row's first alpha entry is its subdomain's plus k times the
    // property's unstable count (the layout of rbase): no per-row load
    const int64_t ab0 = bt.aoff[b];
    const int uc = bt.ucount[p];
    const int64_t pc0 = (int64_t)p * bt.nd + e.layer_off;
    uint32_t rec[NJ];
    float2 ch[NJ];
    float x1[NJ], x2[NJ], x3[NJ], x4[NJ];
    RelaxCoef cf[MODE == kBwdRelax ? NJ : 1];
    AdjCoef af[kBwd ? 1 : NJ];
    RowInfo ri{b, r0 - b * m, p, ab0 + (int64_t)(r0 - b * m) * uc};
    if constexpr (MODE == kBwdRelax) {
      sd_relax_coef<NJ>(bt, v, e, b, p, pl.dout, ab0, uc, cf);
#pragma unroll
      for (int u = 0; u < NJ; ++u) x1[u] = cf[u].vsrc[(int64_t)ri.k * cf[u].vstr];
    } else if constexpr (MODE == kBwdConc) {
      sd_load<MODE>(bt, e, b, p, pl.dout, rec, ch);
    } else {
      sd_adj_coef<NJ>(bt, v, e, b, p, pl.dout, af, x1, x2, x3, x4);
      sd_adj_row_vars<MODE, NJ>(v, ri, af, x1, x2, x3, x4);
      // an l2 ball's first layer: the property's W(1) x0 + b(1) takes the
      // bias's place (every wave is past the previous unit's last epilogue)
      if (e.wx0)
        for (int t = tid; t < pl.dout; t += kSdThreads) bsh[t] = e.wx0[(int64_t)p * e.n + t];
    }
    // the next unit's first row (staged during this unit's last row)
    const int nunit = unit + gridDim.x;
    const int nb = nunit / upb;
    const int nfirst = nunit < n_units ? nb * m + (nunit - nb * upb) * mu : -1;
    const int nprop = MODE == kFwdX && nunit < n_units ? bt.prop[nb] : 0;  // its property
    __syncthreads();  // the unit's first row is staged

    for (int row = r0; row < r1; ++row, par ^= 1) {
      const int nrow = row + 1 < r1 ? row + 1 : nfirst;
      float s1[NI], s2[NI];
      uint32_t g1, g2;
      if (nrow >= 0) {
        if constexpr (MODE == kFwdX) {
          sdx_box<NI>(bt, row + 1 < r1 ? p : nprop, pl.din, s1, s2);
          sdx_words(bt, v, nrow, g1, g2);
        } else {
          in_load<MODE, NI, kSdThreads>(zin, ldi, bt, v, nrow, 0, 0, pl.din, s1, s2, g1, g2);
        }
      }

      if (NJ > 2 || ksp == 1) {
        conv_gemm_row<NT, WG, kSdWaves, true>(pl, zi, zo, wl, mt, kt, ntb, n_ks, n_mt, lane, wave, sct);
      } else {
        const int mtile = wave % n_mt, c = wave / n_mt;
        if (c < ksp) {
          const int np = n_ks >> 2;
          floatx4 acc[NT];
#pragma unroll
          for (int t = 0; t < NT; ++t) acc[t] = floatx4{0.f, 0.f, 0.f, 0.f};
          conv_gemm_tile<NT, WG, true>(pl, zi, wl, mt[mtile * 16 + (lane & 15)].x, kt, uni, kv, (c * np / ksp) * 4,
                                       ((c + 1) * np / ksp) * 4, lane, acc);
#pragma unroll
          for (int t = 0; t < NT; ++t) kpart[(wave * NT + t) * 64 + lane] = acc[t];
        }
        __syncthreads();  // every partial tile is in LDS
        if (wave < n_mt) {  // the tile's sum (chunks in order), scattered
          floatx4 acc[NT];
#pragma unroll
          for (int t = 0; t < NT; ++t) {
            acc[t] = kpart[(wave * NT + t) * 64 + lane];
            for (int cc = 1; cc < ksp; ++cc) acc[t] += kpart[((cc * n_mt + wave) * NT + t) * 64 + lane];
            const int4 ad = sct[(wave * NT + t) * 64 + lane];
            zo[ad.x] = acc[t][0];
            zo[ad.y] = acc[t][1];
            zo[ad.z] = acc[t][2];
            zo[ad.w] = acc[t][3];
          }
        }
      }
      __syncthreads();
      // every wave is past this row's GEMM: zi takes the next row (the rest
      // of a long input row after the epilogue)
      if (nrow >= 0) {
        if constexpr (MODE == kFwdX) {
          // (the next unit's first row: its property's tail of the box first)
          if (row + 1 == r1 && pl.din > kSdThreads * NI) sdx_tail_box<NI>(bt, nprop, pl.din, bxt);
          sdx_stage<NI>(zi, pl, pl.din, s1, s2, g1, g2, bxt);
        } else {
          in_store_at<MODE, NI, kSdThreads>(zi, so, pl.din, s1, s2, g1, g2);
        }
      }

      // ---- epilogue: every operand is in registers.  One wait for every
      // outstanding load here (the row's variables and the staged input have
      // long arrived): the compiler then knows they are ready and issues no
      // wait between the epilogue's stores, which would otherwise each wait
      // for the store before it (stores count against the same counter)
      __builtin_amdgcn_s_waitcnt(kWaitVm0);
      float cst = 0.f, cer = 0.f;
      if constexpr (!kBwd) {
        // the uniform switches are taken once per row, outside the unit loop
        const float rm = e.wx0 ? -v.l2s[row] : 1.f;
        const float* const kb = bsh;
        float* const orow = e.out + (int64_t)row * e.ldo;
        if (v.sat)
          sd_adj_sat<MODE, NJ>(v, zo, pl.dout, rm, kb, orow, row, af);
        else if (v.adam)
          sd_adj_epi<MODE, true, NJ>(bt, v, ri, zo, pl.dout, rm, kb, last ? nullptr : orow, af, x1, x2, x3, x4);
        else
          sd_adj_epi<MODE, false, NJ>(bt, v, ri, zo, pl.dout, rm, kb, last ? nullptr : orow, af, x1, x2, x3, x4);
      }
#pragma unroll
      for (int u = 0; u < (kBwd ? NJ : 0); ++u) {
        const int j = per_row<MODE>(tid + kSdThreads * u);
        const bool ok = j < pl.dout;
        const float a = zo[min(j, pl.dout - 1)];
        if constexpr (MODE == kBwdRelax) {
          if (!ok) continue;
          const RelaxCoef& c = cf[u];
          if (v.acomp && c.cix >= 0) v.acomp[ri.abase + c.cix] = a;
          const float x = x1[u];
          const float t = a >= 0.f ? c.ux * x : c.su;
          const float lam = fmaf(a, c.ca + t, c.sg * x);
          cst = fmaf(fminf(a, 0.f), c.ci, cst);
          cst = fmaf(lam, bsh[j], cst);
          e.out[(int64_t)row * e.ldo + j] = lam;
          if (bt.sw) cer = fmaf(fabsf(lam), bt.sw[pc0 + j], cer);
        } else if (MODE == kBwdConc) {
          if (bt.l2x0) {  // l_p ball: A(0) x0 here, - eps ||A(0)||_q in the final sum
            if (!ok) continue;
            cst = fmaf(a, ch[u].x, cst);
            const float xd = lp_entry(a, bt.lpq, &cer);
            if (v.xdense) v.xdense[(int64_t)row * v.ldx + j] = xd;  // x*'s direction for the adjoint
            continue;
          }
          if (ok) {
            const float tm = conc_term(a, ch[u].x, ch[u].y);
            cst += tm;
            cer = fmaf(bt.sg, fabsf(tm), cer);
          }
          if (v.xpos) {  // x* as sign planes: one 64-bit word per wave
            const uint64_t bp = __ballot(ok && a > 0.f), bn = __ballot(ok && a < 0.f);
            const int w0 = kSdThreads * u + wave * 64;
            if (lane == 0 && w0 < pl.dout) {
              v.xpos[(int64_t)row * bt.w64 + (w0 >> 6)] = bp;
              v.xneg[(int64_t)row * bt.w64 + (w0 >> 6)] = bn;
            }
          }
        }
      }
      if (kBwd) {
        cst = wave_sum(cst);
        cer = wave_sum(cer);
        if (lane == 0) {
          red[par][wave][0] = cst;
          red[par][wave][1] = cer;
        }
      }
      if (MODE != kFwdX && nrow >= 0)
        for (int t0 = kSdThreads * NI; t0 < pl.din; t0 += kSdThreads * NI) {
          in_load<MODE, NI, kSdThreads>(zin, ldi, bt, v, nrow, 0, t0, pl.din, s1, s2, g1, g2);
          in_store<MODE, NI, kSdThreads>(zi, pl, bt, v, nrow, t0, pl.din, s1, s2, g1, g2);
        }
      // the next row's own variables (the unit's status records and chords
      // stay); the next unit's are loaded at its start
      if (row + 1 < r1) {
        ri.k += 1;
        ri.abase += uc;
        if constexpr (MODE == kBwdRelax) {
#pragma unroll
          for (int u = 0; u < NJ; ++u) x1[u] = cf[u].vsrc[(int64_t)ri.k * cf[u].vstr];
        } else if constexpr (!kBwd) {
          sd_adj_row_vars<MODE, NJ>(v, ri, af, x1, x2, x3, x4);
        }
      }
      __syncthreads();
      if (kBwd && tid == 0) {
        float tot = 0.f, ter = 0.f;
#pragma unroll
        for (int w = 0; w < kSdWaves; ++w) {
          tot += red[par][w][0];
          ter += red[par][w][1];
        }
        e.part[(int64_t)e.slot0 * M + row] = tot;
        // rounding-error bound, or the sum of A(0)^2 (l2 ball); with both
        // modes on, the other array's slot gets 0
        float* const p2 = MODE == kBwdConc && bt.l2x0 ? e.psq : (e.perr ? e.perr : e.psq);
        float* const pz = e.perr && e.psq ? (p2 == e.perr ? e.psq : e.perr) : nullptr;
        if (p2) p2[(int64_t)e.slot0 * M + row] = ter;
        if (pz) pz[(int64_t)e.slot0 * M + row] = 0.f;
      }
    }
  }
}

template <int MODE, bool WG>
const void* kernel_nt(int nt) {
  switch (nt) {
    case 1: return reinterpret_cast<const void*>(conv_mm<MODE, 1, WG>);
    case 2: return reinterpret_cast<const void*>(conv_mm<MODE, 2, WG>);
    case 4: return reinterpret_cast<const void*>(conv_mm<MODE, 4, WG>);
    case 8: return reinterpret_cast<const void*>(conv_mm<MODE, 8, WG>);
    default: return nullptr;
  }
}

template <int MODE>
const void* kernel_wg(int nt, bool wg) {
  return wg ? kernel_nt<MODE, true>(nt) : kernel_nt<MODE, false>(nt);
}

const void* kernel_for(int mode, int nt, bool wg) {
  switch (mode) {
    case kBwdRelax: return kernel_wg<kBwdRelax>(nt, wg);
    case kBwdConc: return kernel_wg<kBwdConc>(nt, wg);
    case kFwdX: return kernel_wg<kFwdX>(nt, wg);
    default: return kernel_wg<kFwd>(nt, wg);
  }
}

template <int MODE, bool WG>
int dispatch_wg(const ConvArgs& a, hipStream_t st) {
  // the occupancy query's answer, or two workgroups per CU if it failed
  const dim3 grid(std::min(a.M, a.pl.grid > 0 ? a.pl.grid : 512)), block(256);
#define CVB_CM(NT)                                                                                                \
  case NT:                                                                                                        \
    launch_k(conv_mm<MODE, NT, WG>, grid, block, a.pl.smem, st, a.in, a.ldi, a.pl, a.M, a.last, a.bt, a.v, a.e); \
    return 0;
  switch (a.pl.nt) {
    CVB_CM(1) CVB_CM(2) CVB_CM(4) CVB_CM(8)
    default:
      return -1;
  }
#undef CVB_CM
}

// (NJ, NI) pairs of the subdomain-major kernel instantiated per mode (the
// layer shapes of the CIFAR-sized networks and small test networks)
#define CVB_SD_BWD_RELAX(X) X(2, 2) X(2, 4) X(4, 2) X(4, 4) X(8, 4)
#define CVB_SD_BWD_CONC(X) X(2, 2) X(2, 4) X(6, 4) X(6, 8)
#define CVB_SD_FWD_X(X) X(2, 2) X(4, 4) X(8, 4)
#define CVB_SD_FWD(X) X(2, 2) X(2, 4) X(4, 4) X(4, 8)

template <int MODE, int NT, bool WG>
const void* sd_kernel(int nj, int ni) {
#define CVB_SDK(J, I) \
  if (nj == J && ni == I) return reinterpret_cast<const void*>(conv_sd<MODE, NT, WG, J, I>);
  if constexpr (MODE == kBwdRelax) {
    CVB_SD_BWD_RELAX(CVB_SDK)
  } else if constexpr (MODE == kBwdConc) {
    CVB_SD_BWD_CONC(CVB_SDK)
  } else if constexpr (MODE == kFwdX) {
    CVB_SD_FWD_X(CVB_SDK)
  } else {
    CVB_SD_FWD(CVB_SDK)
  }
#undef CVB_SDK
  return nullptr;
}

template <int MODE>
const void* sd_kernel_for(int nt, bool wg, int nj, int ni) {
  if (nt == 1) return wg ? sd_kernel<MODE, 1, true>(nj, ni) : sd_kernel<MODE, 1, false>(nj, ni);
  if (nt == 2) return wg ? sd_kernel<MODE, 2, true>(nj, ni) : sd_kernel<MODE, 2, false>(nj, ni);
  return nullptr;
}

const void* sd_kernel_mode(int mode, int nt, bool wg, int nj, int ni) {
  switch (mode) {
    case kBwdRelax: return sd_kernel_for<kBwdRelax>(nt, wg, nj, ni);
    case kBwdConc: return sd_kernel_for<kBwdConc>(nt, wg, nj, ni);
    case kFwdX: return sd_kernel_for<kFwdX>(nt, wg, nj, ni);
    default: return sd_kernel_for<kFwd>(nt, wg, nj, ni);
  }
}

// Work-unit size: all of a subdomain's rows when there are few (the
// verification specs), else 16 (the identity specs of the root bounds).
inline int sd_unit_rows(int m) { return m <= 32 ? m : 16; }

template <int MODE, int NT, bool WG>
int launch_sd(const ConvArgs& a, hipStream_t st) {
  const int mu = sd_unit_rows(a.bt.m);
  const int n_units = (a.M / a.bt.m) * ((a.bt.m + mu - 1) / mu);
  const dim3 grid(std::min(n_units, a.pl.grid_sd > 0 ? a.pl.grid_sd : 256)), block(kSdThreads);
#define CVB_SDL(J, I)                                                                                            \
  if (a.pl.nj == J && a.pl.ni == I) {                                                                           \
    launch_k(conv_sd<MODE, NT, WG, J, I>, grid, block, a.pl.smem_sd, st, a.in, a.ldi, a.pl, a.M, a.last, a.bt, a.v, \
             a.e, mu);                                                                                          \
    return 0;                                                                                                   \
  }
  if constexpr (MODE == kBwdRelax) {
    CVB_SD_BWD_RELAX(CVB_SDL)
  } else if constexpr (MODE == kBwdConc) {
    CVB_SD_BWD_CONC(CVB_SDL)
  } else if constexpr (MODE == kFwdX) {
    CVB_SD_FWD_X(CVB_SDL)
  } else {
    CVB_SD_FWD(CVB_SDL)
  }
#undef CVB_SDL
  return -1;
}

template <int MODE>
int dispatch(const ConvArgs& a, hipStream_t st) {
  if (a.M <= 0) return 0;
  // the subdomain-major kernel where an instantiation of this mode holds the
  // plan (a plan built for one mode may be launched in another: over an l2
  // ball the first layer's adjoint reads A(0) rows instead of sign planes),
  // else the row-major one
  // (a pass that stores the adjoint's zbar at upper-chord neurons takes the
  // row-major kernel: the subdomain-major one compiles that store out)
  const bool sd_ok = !(MODE >= kFwdX && a.v.zchord);
  if (sd_ok && a.pl.sd && a.pl.nj > 0 && (a.pl.nt == 1 || a.pl.nt == 2)) {
    const int r = a.pl.nt == 1 ? (a.pl.wg ? launch_sd<MODE, 1, true>(a, st) : launch_sd<MODE, 1, false>(a, st))
                               : (a.pl.wg ? launch_sd<MODE, 2, true>(a, st) : launch_sd<MODE, 2, false>(a, st));
    if (r == 0) return 0;
  }
  return a.pl.wg ? dispatch_wg<MODE, true>(a, st) : dispatch_wg<MODE, false>(a, st);
}

}  // namespace

int conv_plan_smem(const ConvPlan& pl) {
  return ((pl.wg ? 0 : pl.kpad * pl.nt * 16) + ((pl.dinp + 3) & ~3) + pl.dout) * (int)sizeof(float) +
         (pl.mpad + pl.kpad + pl.nt * 16) * (int)sizeof(int4);
}

int conv_plan_grid(int mode, const ConvPlan& pl) {
  const void* k = kernel_for(mode, pl.nt, pl.wg != 0);
  int dev = 0, cus = 0, per = 0;
  if (!k || hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k, 256, pl.smem) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return cus * per;
}

int conv_plan_variant(int mode, ConvPlan& pl, int variant) {
  // 0/1: row-major kernel, 2/3: subdomain-major; odd: weights read from
  // global memory instead of LDS
  const int wg = variant & 1, sd = variant >> 1;
  ConvPlan q = pl;
  q.wg = wg;
  q.smem = conv_plan_smem(q);
  q.grid = conv_plan_grid(mode, q);
  conv_plan_sd(mode, q);
  if (q.smem > 65536 || (sd && (!q.nj || q.smem_sd > 65536 || q.grid_sd <= 0)) || (!sd && q.grid <= 0)) return -1;
  q.sd = sd;
  pl = q;
  return 0;
}

void conv_plan_sd(int mode, ConvPlan& pl) {
  // the smallest instantiated register sizes that hold the row's outputs and inputs
  pl.nj = pl.ni = 0;
  pl.grid_sd = 0;
  pl.sd = 0;
  // (the input prefetch depth ni need not cover the row: the rest is staged
  // after the epilogue)
  int nj = 0, ni = 0;
  for (int c : {2, 4, 6, 8}) {
    if (nj || pl.dout > kSdThreads * c) continue;
    for (int i : {2, 4, 6, 8})
      if (sd_kernel_mode(mode, pl.nt, pl.wg != 0, c, i) && (!ni || pl.din > kSdThreads * ni)) {
        nj = c;
        ni = i;
      }
  }
  if (!nj) return;
  // the first layer's adjoint step reads the sign words of at most 32 chunks of kSdThreads inputs
  if (mode == kFwdX && pl.din > 32 * kSdThreads) return;
  pl.nj = nj;
  pl.ni = ni;
  const void* k = sd_kernel_mode(mode, pl.nt, pl.wg != 0, nj, ni);
  // the plan's LDS, the spare output slot (padded), the scatter table and the bias
  pl.smem_sd = pl.smem + 32 + (pl.mpad >> 4) * pl.nt * 64 * (int)sizeof(int4) +
               (mode == kBwdConc ? 0 : ((pl.dout + 3) & ~3) * (int)sizeof(float)) +
               ((pl.mpad >> 4) < kSdWaves && pl.kpad >= 32 ? kSdWaves * pl.nt * 64 * 16 : 0) +  // split-K partial tiles
               (mode == kFwdX ? 2 * std::max(0, pl.din - kSdThreads * ni) * (int)sizeof(float) : 0);  // box tail
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k, kSdThreads, pl.smem_sd) != hipSuccess) {
    (void)hipGetLastError();
    return;
  }
  pl.grid_sd = cus * per;
  pl.sd = pl.grid_sd > 0 ? 1 : 0;
}

int launch_convt_bwd(int mode, const ConvArgs& a, hipStream_t s) {
  return mode == kBwdConc ? dispatch<kBwdConc>(a, s) : dispatch<kBwdRelax>(a, s);
}

int launch_conv_fwd(int mode, const ConvArgs& a, hipStream_t s) {
  return mode == kFwdX ? dispatch<kFwdX>(a, s) : dispatch<kFwd>(a, s);
}

}  // namespace cvb
