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
// One workgroup per batch row for the dense and convolution layers (the
// row's input in LDS), one wave per row for the top layer.  These kernels
// run once per evaluation in sound mode, not in the optimiser's loop.
#include "common.h"
#include "internal.h"

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

// Back-substitution through conv layer i (transposed convolution): for input
// position (ci, iy, ix), A(i-1) = sum over (co, ky, kx) with oy = (iy + pad -
// ky) / stride and ox likewise whole and inside the output plane of
// Lambda(i)[co, oy, ox] W[co, ci, ky, kx], in double.
// The weights are staged in LDS after the row when they fit (w_lds), else
// read from global memory; the same values and order either way.
__global__ __launch_bounds__(256) void conv64_k(Pass64 q, Lay64 y, ConvGeom g, int w_lds) {
  extern __shared__ double lam_s[];
  __shared__ double red[4];
  const int row = blockIdx.x;
  const RowInfo ri = row_info(q.bt, row);
  float* const w_s = reinterpret_cast<float*>(lam_s + y.K);
  const float* const W = w_lds ? w_s : y.W;
  for (int k = threadIdx.x; k < y.K; k += 256) lam_s[k] = y.in[(int64_t)row * y.ldi + k];
  if (w_lds)
    for (int t = threadIdx.x; t < g.co * g.ci * g.k * g.k; t += 256) w_s[t] = y.W[t];
  __syncthreads();
  double cst = 0.0, err = 0.0, sq = 0.0;
  for (int j = threadIdx.x; j < y.N; j += 256) {
    const int ci = j / (g.hi * g.wi), rem = j - ci * g.hi * g.wi;
    const int iy = rem / g.wi, ix = rem - iy * g.wi;
    double a = 0.0;
    // the taps with iy + p - ky a non-negative multiple of the stride, in
    // ascending ky (then kx, then co): ky = ry, ry + s, ... and oy = oy0, oy0 - 1, ...
    const int ry = (iy + g.p) % g.s, rx = (ix + g.p) % g.s;
    const int oy0 = (iy + g.p - ry) / g.s, ox0 = (ix + g.p - rx) / g.s;
    for (int ky = ry, oy = oy0; ky < g.k && oy >= 0; ky += g.s, --oy) {
      if (oy >= g.ho) continue;
      for (int kx = rx, ox = ox0; kx < g.k && ox >= 0; kx += g.s, --ox) {
        if (ox >= g.wo) continue;
        for (int co = 0; co < g.co; ++co)
          a += lam_s[(co * g.ho + oy) * g.wo + ox] * (double)W[((co * g.ci + ci) * g.k + ky) * g.k + kx];
      }
    }
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
  if (q.bt.n_rows > 0) launch_k(dense64_k, (unsigned)q.bt.n_rows, 256, (uint32_t)(y.K * sizeof(double)), s, q, y);
}

void launch_conv64(const Pass64& q, const Lay64& y, const ConvGeom& g, hipStream_t s) {
  if (q.bt.n_rows <= 0) return;
  const size_t row_b = (size_t)y.K * sizeof(double), w_b = (size_t)g.co * g.ci * g.k * g.k * sizeof(float);
  const int w_lds = row_b + w_b <= 48 * 1024 ? 1 : 0;
  launch_k(conv64_k, (unsigned)q.bt.n_rows, 256, (uint32_t)(row_b + (w_lds ? w_b : 0)), s, q, y, g, w_lds);
}

void launch_finalize64(const Pass64& q, const Fin64& f, hipStream_t s) {
  if (q.bt.n_rows > 0) launch_k(finalize64_k, (unsigned)((q.bt.n_rows + 255) / 256), 256, 0, s, q, f);
}

}  // namespace cvb
