// Sound-mode evaluation of the bound in float64 (gfx950).
//
// The same recursion as the float32 kernels (Theorem 3.1, Eq. definition_A:
// Lambda(i) = A(i) D(i) + beta^T S(i), A(i-1) = Lambda(i) W(i), the constants
// A lowerb + Lambda b, and the concretisation of A(0) over the input set),
// carried out in double: the specification merged into the last layer, every
// product, the relaxation (with the chord u/(u-l), -ul/(u-l) formed in double
// from the float bounds), the constants and the concretisation.  Each kernel
// also accumulates a rigorous bound on its own float64 rounding error, per
// row (weights per neuron from the host analysis, with the unit roundoff of
// double), and the final sum subtracts it and rounds the result down to
// float: the reported bound lies below the exact bound of the same relaxation
// by that margin (about 1e-13 of the terms' magnitudes) plus one float ulp.
//
// One workgroup per batch row for the dense and convolution layers (four
// rows per workgroup for dense layers on large batches; the rows' inputs in
// LDS), one wave per row for the top layer.  These kernels run once per evaluation in sound
// mode, not in the optimiser's loop.
#include "common.h"
#include "internal.h"

#include <type_traits>
#include <utility>

namespace cvb {

namespace {

__device__ __forceinline__ double wave_sum_d(double x) {
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

// Sum over a 256-thread block, returned to thread 0 (red: 4 doubles of LDS).
__device__ __forceinline__ double block_sum_d(double x, double* red) {
  x = wave_sum_d(x);
  __syncthreads();  // red may still be read from the previous call
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = x;
  __syncthreads();
  return threadIdx.x == 0 ? (red[0] + red[1]) + (red[2] + red[3]) : 0.0;
}

// Relaxation of one neuron in double (Lemma 2.1 cases, the split term); adds
// A lowerb + Lambda b to cst and |Lambda| sw to err; returns Lambda.
__device__ __forceinline__ double relax64(const Pass64& q, const RowInfo& ri, uint32_t rec, int64_t pc, double a,
                                          double bias, double& cst, double& err) {
  const uint32_t kind = rec & kKindMask;
  double lam = 0.0;
  if (kind == kActive) {
    lam = a;
  } else if (kind == kUnstable) {
    if (a >= 0.0) {
      const int64_t ai = ri.abase + (rec & kCidxMask);
      lam = (double)(q.alpha ? q.alpha[ai] : q.bt.adef[pc]) * a;
    } else {
      const double l = q.l[pc], u = q.u[pc];
      const double den = u - l;  // exact: both are floats
      lam = a * (u / den);
      cst += a * (-(u * l) / den);
    }
  } else if (kind == kSplit) {
    const double be = q.beta[(int64_t)(rec & kSplitMask) * q.bt.m + ri.k];
    lam = (rec & kSidePos) ? a - be : be;
  }
  cst += lam * bias;
  err += fabs(lam) * (double)q.sw[pc];
  return lam;
}

// Concretisation of one input coordinate: the box minimum, or over an l2 ball
// A x0 (with A^2 into sq).
__device__ __forceinline__ void conc64(const Pass64& q, int p, int j, double a, double& cst, double& err,
                                       double& sq) {
  const int64_t pb = (int64_t)p * q.bt.d0 + j;
  if (q.bt.l2x0) {
    cst += a * (double)q.bt.l2x0[pb];
    sq += a * a;
    return;
  }
  const double tm = fmin(a * (double)q.bt.xlo[pb], a * (double)q.bt.xhi[pb]);
  cst += tm;
  err += q.sg * fabs(tm);
}

// relax64 / conc64 over a thread's outputs j0 + 256 u (u < kC, those below
// N), in ascending j: the operands are loaded first, in two rounds of
// independent loads (the status words, then what they select), and each
// neuron then takes relax64's (conc64's) arithmetic in the same order.
template <int kC>
__device__ __forceinline__ void epi64(const Pass64& q, const RowInfo& ri, const Lay64& y, int row, int j0,
                                      const double (&a)[kC], double& cst, double& err, double& sq) {
  if (y.conc) {
    float x0[kC], x1[kC];
#pragma unroll
    for (int u = 0; u < kC; ++u) {
      const int j = j0 + 256 * u;
      x0[u] = x1[u] = 0.f;
      if (j < y.N) {
        const int64_t pb = (int64_t)ri.p * q.bt.d0 + j;
        if (q.bt.l2x0) {
          x0[u] = q.bt.l2x0[pb];
        } else {
          x0[u] = q.bt.xlo[pb];
          x1[u] = q.bt.xhi[pb];
        }
      }
    }
    // local copies, all three written back, so that neither branch updates
    // its sum through memory
    double c = cst, e = err, s2 = sq;
    if (q.bt.l2x0) {
#pragma unroll
      for (int u = 0; u < kC; ++u) {
        if (j0 + 256 * u >= y.N) continue;
        c += a[u] * (double)x0[u];
        s2 += a[u] * a[u];
      }
    } else {
#pragma unroll
      for (int u = 0; u < kC; ++u) {
        if (j0 + 256 * u >= y.N) continue;
        const double tm = fmin(a[u] * (double)x0[u], a[u] * (double)x1[u]);
        c += tm;
        e += q.sg * fabs(tm);
      }
    }
    cst = c;
    err = e;
    sq = s2;
    return;
  }
  uint32_t rec[kC];
#pragma unroll
  for (int u = 0; u < kC; ++u) {
    const int j = j0 + 256 * u;
    rec[u] = j < y.N ? q.bt.status[(int64_t)ri.b * q.bt.nd + y.layer_off + j] : 0u;
  }
  // o0: alpha (unstable, A >= 0), l (unstable, A < 0) or beta (split); o1: u
  float o0[kC], o1[kC], swv[kC], bv[kC];
#pragma unroll
  for (int u = 0; u < kC; ++u) {
    const int j = j0 + 256 * u;
    o0[u] = o1[u] = swv[u] = bv[u] = 0.f;
    if (j >= y.N) continue;
    const int64_t pc = (int64_t)ri.p * q.bt.nd + y.layer_off + j;
    swv[u] = q.sw[pc];
    bv[u] = y.bias[j];
    const uint32_t kind = rec[u] & kKindMask;
    if (kind == kUnstable) {
      if (a[u] >= 0.0) {
        o0[u] = q.alpha ? q.alpha[ri.abase + (rec[u] & kCidxMask)] : q.bt.adef[pc];
      } else {
        o0[u] = q.l[pc];
        o1[u] = q.u[pc];
      }
    } else if (kind == kSplit) {
      o0[u] = q.beta[(int64_t)(rec[u] & kSplitMask) * q.bt.m + ri.k];
    }
  }
#pragma unroll
  for (int u = 0; u < kC; ++u) {
    const int j = j0 + 256 * u;
    if (j >= y.N) continue;
    const uint32_t kind = rec[u] & kKindMask;
    const double av = a[u];
    double lam = 0.0;
    if (kind == kActive) {
      lam = av;
    } else if (kind == kUnstable) {
      if (av >= 0.0) {
        lam = (double)o0[u] * av;
      } else {
        const double l = o0[u], uu = o1[u];
        const double den = uu - l;  // exact: both are floats
        lam = av * (uu / den);
        cst += av * (-(uu * l) / den);
      }
    } else if (kind == kSplit) {
      const double be = o0[u];
      lam = (rec[u] & kSidePos) ? av - be : be;
    }
    cst += lam * (double)bv[u];
    err += fabs(lam) * (double)swv[u];
    y.out[(int64_t)row * y.ldo + j] = lam;
  }
}

// The top ReLU layer: A(L-1) = C_p W(L) in double (general specification) or
// the exact rows +-W(L) (identity specification, as float rows CW), relaxed
// (or concretised when there is no ReLU layer).  One wave per row.
__global__ __launch_bounds__(256) void top64_k(Pass64 q, Top64 t) {
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= q.bt.n_rows) return;
  const RowInfo ri = row_info(q.bt, row);
  double cst = 0.0, err = 0.0, sq = 0.0;
  double c0;
  const float* crow = t.C ? t.C + ((int64_t)ri.p * q.bt.m + ri.k) * t.dL : nullptr;
  if (crow) {
    c0 = 0.0;
    for (int o = 0; o < t.dL; ++o) c0 += (double)crow[o] * (double)t.bL[o];
  } else {
    c0 = (double)t.Cb[ri.p * t.cb_pstride + ri.k];
  }
  for (int j = lane; j < t.n; j += 64) {
    double a;
    if (crow) {
      a = 0.0;
      for (int o = 0; o < t.dL; ++o) a += (double)crow[o] * (double)t.WL[(int64_t)o * t.ldw + j];
    } else {
      a = (double)t.CW[ri.p * t.cw_pstride + (int64_t)ri.k * t.ldcw + j];
    }
    if (t.conc) {
      conc64(q, ri.p, j, a, cst, err, sq);
    } else {
      const int64_t pc = (int64_t)ri.p * q.bt.nd + t.layer_off + j;
      const uint32_t rec = q.bt.status[(int64_t)ri.b * q.bt.nd + t.layer_off + j];
      t.out[(int64_t)row * t.ldo + j] = relax64(q, ri, rec, pc, a, (double)t.bias[j], cst, err);
    }
  }
  cst = wave_sum_d(cst);
  err = wave_sum_d(err);
  sq = wave_sum_d(sq);
  if (lane == 0) {
    q.part[row] = cst + c0;
    q.perr[row] = err + (double)t.err0[ri.p * q.bt.m + ri.k];
    if (q.psq) q.psq[row] = sq;
  }
}

// Back-substitution through dense layer i: A(i-1)_j = sum_k Lambda(i)_k W(i)_kj
// in double, then the relaxation of layer i-1 (or the concretisation).
__global__ __launch_bounds__(256) void dense64_k(Pass64 q, Lay64 y) {
  extern __shared__ double lam_s[];
  __shared__ double red[4];
  const int row = blockIdx.x;
  const RowInfo ri = row_info(q.bt, row);
  for (int k = threadIdx.x; k < y.K; k += 256) lam_s[k] = y.in[(int64_t)row * y.ldi + k];
  __syncthreads();
  double cst = 0.0, err = 0.0, sq = 0.0;
  for (int j = threadIdx.x; j < y.N; j += 256) {
    double a = 0.0;
    for (int k = 0; k < y.K; ++k) a += lam_s[k] * (double)y.W[(int64_t)k * y.ldw + j];
    if (y.conc) {
      conc64(q, ri.p, j, a, cst, err, sq);
    } else {
      const int64_t pc = (int64_t)ri.p * q.bt.nd + y.layer_off + j;
      const uint32_t rec = q.bt.status[(int64_t)ri.b * q.bt.nd + y.layer_off + j];
      y.out[(int64_t)row * y.ldo + j] = relax64(q, ri, rec, pc, a, (double)y.bias[j], cst, err);
    }
  }
  const double c = block_sum_d(cst, red), e = block_sum_d(err, red), s2 = block_sum_d(sq, red);
  if (threadIdx.x == 0) {
    q.part[(int64_t)y.slot * q.bt.n_rows + row] = c;
    q.perr[(int64_t)y.slot * q.bt.n_rows + row] = e;
    if (q.psq) q.psq[(int64_t)y.slot * q.bt.n_rows + row] = s2;
  }
}

// The same for kDenseRows consecutive rows per workgroup (rpb, all of them
// in LDS), so that each weight read serves every one of them, on large
// batches; each row's sums keep the one-row order.
constexpr int kDenseRows = 4;
__global__ __launch_bounds__(256) void dense64_rows_k(Pass64 q, Lay64 y, int rpb) {
  extern __shared__ double lam_s[];
  __shared__ double red[4];
  const int row0 = blockIdx.x * rpb;
  const int nr = min(rpb, q.bt.n_rows - row0);
  const int tot = nr * y.K;
  for (int t0 = threadIdx.x; t0 < tot; t0 += 256 * 8) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int t = t0 + 256 * u, r = t / y.K;
      v[u] = t < tot ? y.in[(int64_t)(row0 + r) * y.ldi + (t - r * y.K)] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (t0 + 256 * u < tot) lam_s[t0 + 256 * u] = v[u];
  }
  __syncthreads();
  double cst[kDenseRows], err[kDenseRows], sq[kDenseRows];
  RowInfo ri[kDenseRows];
#pragma unroll
  for (int r = 0; r < kDenseRows; ++r) {
    cst[r] = err[r] = sq[r] = 0.0;
    if (r < nr) ri[r] = row_info(q.bt, row0 + r);
  }
  constexpr int kC = 2;
  for (int j0 = threadIdx.x; j0 < y.N; j0 += 256 * kC) {
    double a[kDenseRows][kC];
#pragma unroll
    for (int r = 0; r < kDenseRows; ++r)
#pragma unroll
      for (int u = 0; u < kC; ++u) a[r][u] = 0.0;
    for (int k = 0; k < y.K; ++k) {
      double w[kC];
#pragma unroll
      for (int u = 0; u < kC; ++u) {
        const int j = j0 + 256 * u;
        w[u] = j < y.N ? (double)y.W[(int64_t)k * y.ldw + j] : 0.0;
      }
#pragma unroll
      for (int r = 0; r < kDenseRows; ++r) {
        if (r < nr) {
          const double l = lam_s[r * y.K + k];
#pragma unroll
          for (int u = 0; u < kC; ++u) a[r][u] += l * w[u];
        }
      }
    }
#pragma unroll
    for (int r = 0; r < kDenseRows; ++r)
      if (r < nr) epi64<kC>(q, ri[r], y, row0 + r, j0, a[r], cst[r], err[r], sq[r]);
  }
#pragma unroll
  for (int r = 0; r < kDenseRows; ++r) {
    if (r < nr) {  // nr is uniform over the workgroup
      const double c = block_sum_d(cst[r], red), e = block_sum_d(err[r], red), s2 = block_sum_d(sq[r], red);
      if (threadIdx.x == 0) {
        const int64_t o = (int64_t)y.slot * q.bt.n_rows + row0 + r;
        q.part[o] = c;
        q.perr[o] = e;
        if (q.psq) q.psq[o] = s2;
      }
    }
  }
}

// a[U] = f(U) for the constant indices U (the array stays in registers).
template <int kC, class F, int... U>
__device__ __forceinline__ void fill_seq(double (&a)[kC], F f, std::integer_sequence<int, U...>) {
  ((a[U] = f(U)), ...);
}

// A(i-1) at input position j of a conv layer (0 for j >= N): the taps with
// iy + p - ky a non-negative multiple of the stride, in ascending ky (then kx,
// then co): ky = ry, ry + s, ... and oy = oy0, oy0 - 1, ...
__device__ __forceinline__ double tap_sum64(const double* lam_s, const float* W, const ConvGeom& g, int N, int j) {
  if (j >= N) return 0.0;
  const int ci = j / (g.hi * g.wi), rem = j - ci * g.hi * g.wi;
  const int iy = rem / g.wi, ix = rem - iy * g.wi;
  const int ry = (iy + g.p) % g.s, rx = (ix + g.p) % g.s;
  const int oy0 = (iy + g.p - ry) / g.s, ox0 = (ix + g.p - rx) / g.s;
  double acc = 0.0;
  for (int ky = ry, oy = oy0; ky < g.k && oy >= 0; ky += g.s, --oy) {
    if (oy >= g.ho) continue;
    for (int kx = rx, ox = ox0; kx < g.k && ox >= 0; kx += g.s, --ox) {
      if (ox >= g.wo) continue;
#pragma unroll 8
      for (int co = 0; co < g.co; ++co)
        acc += lam_s[(co * g.ho + oy) * g.wo + ox] * (double)W[((co * g.ci + ci) * g.k + ky) * g.k + kx];
    }
  }
  return acc;
}

constexpr int kC64 = 8;  // outputs per thread per pass of the conv kernel

// The outputs of one row, with the weights W in LDS or in global memory (a
// separate instance for each, so that LDS weights are read as LDS).
template <int kC>
__device__ __forceinline__ void conv64_row(const Pass64& q, const Lay64& y, const ConvGeom& g, const RowInfo& ri,
                                           int row, const double* lam_s, const float* W, double& cst, double& err,
                                           double& sq) {
  for (int j0 = threadIdx.x; j0 < y.N; j0 += 256 * kC) {
    double a[kC];
    fill_seq(a, [&](int u) { return tap_sum64(lam_s, W, g, y.N, j0 + 256 * u); }, std::make_integer_sequence<int, kC>{});
    epi64<kC>(q, ri, y, row, j0, a, cst, err, sq);
  }
}

// The outputs of one row when the plane size hi wi divides 256 (DCI = 256 /
// (hi wi)): a thread's outputs j0 + 256 u then sit at one position, in
// channels ci0 + DCI u, and share their taps, so each Lambda value read from
// LDS serves all kC of them.  wt holds the weights in LDS as [co][ky][kx][cip]
// (input channel innermost, zero past ci).  Each output's sum keeps the order
// of tap_sum64.
template <int kC, int DCI>
__device__ __forceinline__ void conv64_row_pos(const Pass64& q, const Lay64& y, const ConvGeom& g,
                                               const RowInfo& ri, int row, const double* lam_s, const float* wt,
                                               int cip, double& cst, double& err, double& sq) {
  constexpr int hw = 256 / DCI;
  for (int j0 = threadIdx.x; j0 < y.N; j0 += 256 * kC) {
    const int ci0 = j0 / hw, pos = j0 - ci0 * hw;
    const int iy = pos / g.wi, ix = pos - iy * g.wi;
    const int ry = (iy + g.p) % g.s, rx = (ix + g.p) % g.s;
    const int oy0 = (iy + g.p - ry) / g.s, ox0 = (ix + g.p - rx) / g.s;
    double a[kC];
#pragma unroll
    for (int u = 0; u < kC; ++u) a[u] = 0.0;
    for (int ky = ry, oy = oy0; ky < g.k && oy >= 0; ky += g.s, --oy) {
      if (oy >= g.ho) continue;
      for (int kx = rx, ox = ox0; kx < g.k && ox >= 0; kx += g.s, --ox) {
        if (ox >= g.wo) continue;
        const float* wp = wt + (ky * g.k + kx) * cip + ci0;
#pragma unroll 2
        for (int co = 0; co < g.co; ++co) {
          const double l = lam_s[(co * g.ho + oy) * g.wo + ox];
          const float* w = wp + co * g.k * g.k * cip;
#pragma unroll
          for (int u = 0; u < kC; ++u) a[u] += l * (double)w[DCI * u];
        }
      }
    }
    epi64<kC>(q, ri, y, row, j0, a, cst, err, sq);
  }
}

// The outputs of one row for a 3-channel input of 1024 positions (32x32):
// N = 3072, so a thread's outputs j0 + 256 u (u < 12, one pass) sit at four
// positions j0 + 256 g, each in all three channels (u = g + 4 c).  Each
// Lambda value read from LDS serves the three channels of its position; wt
// holds the weights as [co][ky][kx][3].  Each output's sum keeps the order of
// tap_sum64, and the epilogue takes the outputs in ascending j as before.
__device__ __forceinline__ void conv64_row_rgb(const Pass64& q, const Lay64& y, const ConvGeom& g,
                                               const RowInfo& ri, int row, const double* lam_s, const float* wt,
                                               double& cst, double& err, double& sq) {
  constexpr int P = 4, C = 3, kC = P * C;
  const int j0 = threadIdx.x;
  double a[kC];
#pragma unroll
  for (int u = 0; u < kC; ++u) a[u] = 0.0;
  // one position (a compile-time gi, so that a stays in registers)
  auto position = [&](auto gic) {
    constexpr int gi = decltype(gic)::value;
    const int pos = j0 + 256 * gi;
    const int iy = pos / g.wi, ix = pos - iy * g.wi;
    const int ry = (iy + g.p) % g.s, rx = (ix + g.p) % g.s;
    const int oy0 = (iy + g.p - ry) / g.s, ox0 = (ix + g.p - rx) / g.s;
    for (int ky = ry, oy = oy0; ky < g.k && oy >= 0; ky += g.s, --oy) {
      if (oy >= g.ho) continue;
      for (int kx = rx, ox = ox0; kx < g.k && ox >= 0; kx += g.s, --ox) {
        if (ox >= g.wo) continue;
        const float* wp = wt + (ky * g.k + kx) * C;
#pragma unroll 2
        for (int co = 0; co < g.co; ++co) {
          const double l = lam_s[(co * g.ho + oy) * g.wo + ox];
          const float* w = wp + co * g.k * g.k * C;
#pragma unroll
          for (int c = 0; c < C; ++c) a[gi + P * c] += l * (double)w[c];
        }
      }
    }
  };
  position(std::integral_constant<int, 0>{});
  position(std::integral_constant<int, 1>{});
  position(std::integral_constant<int, 2>{});
  position(std::integral_constant<int, 3>{});
  epi64<kC>(q, ri, y, row, j0, a, cst, err, sq);
}

// Back-substitution through conv layer i (transposed convolution): for input
// position (ci, iy, ix), A(i-1) = sum over (co, ky, kx) with oy = (iy + pad -
// ky) / stride and ox likewise whole and inside the output plane of
// Lambda(i)[co, oy, ox] W[co, ci, ky, kx], in double.
// The weights are staged in LDS after the row when they fit (w_lds: as
// stored, or in the position-blocked layout of conv64_row_pos when the plane
// size divides 256, or of conv64_row_rgb for a 3x32x32 input), else read
// from global memory; the same values and the same order of every sum in
// every case.
template <int w_lds>
__global__ __launch_bounds__(256) void conv64_k(Pass64 q, Lay64 y, ConvGeom g) {
  extern __shared__ double lam_s[];
  __shared__ double red[4];
  const int row = blockIdx.x;
  const RowInfo ri = row_info(q.bt, row);
  float* const w_s = reinterpret_cast<float*>(lam_s + ((y.K + 1) & ~1));
  for (int k0 = threadIdx.x; k0 < y.K; k0 += 256 * 8) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int k = k0 + 256 * u;
      v[u] = k < y.K ? y.in[(int64_t)row * y.ldi + k] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (k0 + 256 * u < y.K) lam_s[k0 + 256 * u] = v[u];
  }
  // w_lds: 1 the weights as stored, 2 the position-blocked layout of
  // conv64_row_pos with dci = 256 / (hi wi) and cip channels, 3 that layout
  // with cip = 3 for conv64_row_rgb, 0 global memory
  const int dci = w_lds == 2 ? 256 / (g.hi * g.wi) : 0, cip = w_lds == 3 ? 3 : g.ci + dci * kC64;
  if constexpr (w_lds == 1) {
    for (int t = threadIdx.x; t < g.co * g.ci * g.k * g.k; t += 256) w_s[t] = y.W[t];
  } else if constexpr (w_lds >= 2) {
    for (int t = threadIdx.x; t < g.co * g.k * g.k * cip; t += 256) {
      const int c = t % cip, r = t / cip, kx = r % g.k, r2 = r / g.k, ky = r2 % g.k, co = r2 / g.k;
      w_s[t] = c < g.ci ? y.W[((co * g.ci + c) * g.k + ky) * g.k + kx] : 0.f;
    }
  }
  __syncthreads();
  double cst = 0.0, err = 0.0, sq = 0.0;
  if constexpr (w_lds == 3) {
    conv64_row_rgb(q, y, g, ri, row, lam_s, w_s, cst, err, sq);
  } else if constexpr (w_lds == 2) {
    if (dci == 1) conv64_row_pos<kC64, 1>(q, y, g, ri, row, lam_s, w_s, cip, cst, err, sq);
    else if (dci == 2) conv64_row_pos<kC64, 2>(q, y, g, ri, row, lam_s, w_s, cip, cst, err, sq);
    else if (dci == 4) conv64_row_pos<kC64, 4>(q, y, g, ri, row, lam_s, w_s, cip, cst, err, sq);
    else conv64_row_pos<kC64, 8>(q, y, g, ri, row, lam_s, w_s, cip, cst, err, sq);
  } else if constexpr (w_lds == 1) {
    conv64_row<kC64>(q, y, g, ri, row, lam_s, w_s, cst, err, sq);
  } else {
    conv64_row<kC64>(q, y, g, ri, row, lam_s, y.W, cst, err, sq);
  }
  const double c = block_sum_d(cst, red), e = block_sum_d(err, red), s2 = block_sum_d(sq, red);
  if (threadIdx.x == 0) {
    q.part[(int64_t)y.slot * q.bt.n_rows + row] = c;
    q.perr[(int64_t)y.slot * q.bt.n_rows + row] = e;
    if (q.psq) q.psq[(int64_t)y.slot * q.bt.n_rows + row] = s2;
  }
}

// Round a double down to a float (the largest float <= x).
__device__ __forceinline__ float down_f(double x) {
  float f = (float)x;
  if ((double)f > x) f = nextafterf(f, -INFINITY);
  return f;
}

// lb = (sum of the constants) - (margin), rounded down to float.  The margin
// is the sum of the rounding-error partials scaled by `scale` (their own
// summation), plus, over an l2 ball, eps ||A(0)||_2 (taken as an upper bound:
// the sum of squares and the square root inflated by `ball`, which also
// covers the float64 rounding of the A(0) x0 sum, bounded by ball ||A(0)||_2
// ||x0||_2), plus the rounding of the final subtraction.
__global__ __launch_bounds__(256) void finalize64_k(Pass64 q, Fin64 f) {
  const int row = blockIdx.x * 256 + threadIdx.x;
  if (row >= q.bt.n_rows) return;
  double tot = 0.0, err = 0.0, s2 = 0.0;
  for (int t = 0; t < f.n_used; ++t) {
    tot += q.part[(int64_t)t * q.bt.n_rows + row];
    err += q.perr[(int64_t)t * q.bt.n_rows + row];
    if (q.psq) s2 += q.psq[(int64_t)t * q.bt.n_rows + row];
  }
  double margin = err * f.scale;
  if (q.psq) {
    const int p = q.bt.prop[row / q.bt.m];
    const double nrm = sqrt(s2) * (1.0 + f.ball);
    tot -= (double)q.bt.l2eps[p] * nrm;
    margin += ((double)q.bt.l2eps[p] + (double)f.x0n[p]) * nrm * f.ball;
  }
  const double d = tot - margin;
  const float lbv = down_f(d - fabs(d) * 0x1p-52 - 0x1p-1000);
  if (f.lb) f.lb[row] = lbv;
  if (f.best) f.best[row] = f.first ? lbv : fmaxf(f.best[row], lbv);
}

}  // namespace

void launch_top64(const Pass64& q, const Top64& t, hipStream_t s) {
  if (q.bt.n_rows > 0) launch_k(top64_k, (unsigned)((q.bt.n_rows + 3) / 4), 256, 0, s, q, t);
}

void launch_dense64(const Pass64& q, const Lay64& y, hipStream_t s) {
  if (q.bt.n_rows <= 0) return;
  // several rows per workgroup on batches that still give 4096+ workgroups,
  // while the rows fit in 64 KB of LDS; else one (K <= 8192 always fits)
  const int rpb = std::min(kDenseRows, (int)(64 * 1024 / (std::max(y.K, 1) * sizeof(double))));
  if (q.bt.n_rows >= 4096 * kDenseRows && rpb == kDenseRows)
    launch_k(dense64_rows_k, (unsigned)((q.bt.n_rows + rpb - 1) / rpb), 256, (uint32_t)(rpb * y.K * sizeof(double)),
             s, q, y, rpb);
  else
    launch_k(dense64_k, (unsigned)q.bt.n_rows, 256, (uint32_t)(y.K * sizeof(double)), s, q, y);
}

void launch_conv64(const Pass64& q, const Lay64& y, const ConvGeom& g, hipStream_t s) {
  if (q.bt.n_rows <= 0) return;
  const size_t row_b = (size_t)((y.K + 1) & ~1) * sizeof(double), w_b = (size_t)g.co * g.ci * g.k * g.k * sizeof(float);
  const int hw = g.hi * g.wi;
  const size_t wt_b = (size_t)g.co * g.k * g.k * (g.ci + (hw > 0 ? 256 / hw : 0) * kC64) * sizeof(float);
  int w_lds = 0;
  size_t lds = row_b;
  if (hw == 1024 && g.ci == 3 && y.N == 3 * 1024 && row_b + w_b <= 48 * 1024) {
    w_lds = 3;  // the [co][ky][kx][3] layout holds the same number of weights
    lds += w_b;
  } else if (hw >= 32 && 256 % hw == 0 && y.N == g.ci * hw && row_b + wt_b <= 48 * 1024) {
    w_lds = 2;
    lds += wt_b;
  } else if (row_b + w_b <= 48 * 1024) {
    w_lds = 1;
    lds += w_b;
  }
  const unsigned nb = (unsigned)q.bt.n_rows;
  if (w_lds == 3) launch_k(conv64_k<3>, nb, 256, (uint32_t)lds, s, q, y, g);
  else if (w_lds == 2) launch_k(conv64_k<2>, nb, 256, (uint32_t)lds, s, q, y, g);
  else if (w_lds == 1) launch_k(conv64_k<1>, nb, 256, (uint32_t)lds, s, q, y, g);
  else launch_k(conv64_k<0>, nb, 256, (uint32_t)lds, s, q, y, g);
}

void launch_finalize64(const Pass64& q, const Fin64& f, hipStream_t s) {
  if (q.bt.n_rows > 0) launch_k(finalize64_k, (unsigned)((q.bt.n_rows + 255) / 256), 256, 0, s, q, f);
}

}  // namespace cvb
