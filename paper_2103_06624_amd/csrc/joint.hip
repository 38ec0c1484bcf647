// Kernels of the joint optimisation of intermediate bounds (Sec. 3.3, Eq.
// opt_non_convex): per-subdomain relaxation tables refreshed from the current
// bounds, the clip of computed bounds by the root bounds, the broadcast of the
// per-layer shared variables to the rows of an intermediate-bound pass and the
// weighted reduction of the rows' gradients back onto them, and the gradient
// of the bound with respect to the intermediate bounds themselves.
#include "common.h"
#include "internal.h"

namespace cvb {

namespace {

inline unsigned nblk(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

constexpr float kTie = 1e-4f;  // relative width of a tie between a computed and a root bound

// status / chord of columns [0, nd_x) of handle X (row stride nd_x) from the
// current bounds (row stride nd).  A root-unstable unsplit neuron is active
// when l >= 0, inactive when u <= 0, else unstable with its root chord index;
// every other word keeps its root value (splits decide their own neurons).
__global__ void refresh_k(uint32_t* status, const uint32_t* __restrict__ status0, float2* chord,
                          const float* __restrict__ lcur, const float* __restrict__ ucur, int B, int nd_x, int nd) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)B * nd_x) return;
  const int b = (int)(i / nd_x);
  const int c = (int)(i - (int64_t)b * nd_x);
  const uint32_t r0 = status0[i];
  uint32_t r = r0;
  float2 ch = make_float2(0.f, 0.f);
  if ((r0 & kKindMask) == kUnstable) {
    const float l = lcur[(int64_t)b * nd + c], u = ucur[(int64_t)b * nd + c];
    if (l >= 0.f) {
      r = kActive;
    } else if (u <= 0.f) {
      r = kInactive;
    } else {
      // upper chord of ReLU on [l, u] (Lemma 2.1)
      const float den = u - l;
      ch = make_float2(u / den, -u * l / den);
    }
  }
  status[i] = r;
  chord[i] = ch;
}

// layer bounds from the rows of an intermediate pass ([B][2d]: z lower
// bounds, then bounds of -z): the tighter of the computed and the root bound;
// ml / mu mark where the gradient follows the computed bound -- unless it is
// looser than the root's by more than kTie max(1, |root|) (a tie is decided
// for the computed bound, whatever the rounding)
__global__ void clip_k(const float* __restrict__ lb, int d, int off, const float* __restrict__ lroot,
                       const float* __restrict__ uroot, float* lcur, float* ucur, uint8_t* ml, uint8_t* mu, int B,
                       int nd) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)B * d) return;
  const int b = (int)(i / d);
  const int j = (int)(i - (int64_t)b * d);
  const int64_t c = (int64_t)b * nd + off + j;
  const float ln = lb[(int64_t)b * 2 * d + j], un = -lb[(int64_t)b * 2 * d + d + j];
  const float lr = lroot[c], ur = uroot[c];
  lcur[c] = fmaxf(ln, lr);
  ucur[c] = fminf(un, ur);
  ml[c] = ln >= lr - kTie * fmaxf(fabsf(lr), 1.f);
  mu[c] = un <= ur + kTie * fmaxf(fabsf(ur), 1.f);
}

// alpha' rows of the pass: row (b, k) takes the shared block of its side
// (k >= d: the upper bounds); the shared blocks of b start at aoff[b] / d
__global__ void bcast_alpha_k(float* arow, const float* __restrict__ ash, Batch bt, int d) {
  const int r = blockIdx.x;
  const int b = r / bt.m, k = r - b * bt.m;
  const int uc = bt.ucount[b];
  const float* src = ash + bt.aoff[b] / d + (k >= d ? uc : 0);
  float* dst = arow + bt.rbase[r];
  for (int c = threadIdx.x; c < uc; c += blockDim.x) dst[c] = src[c];
}

__global__ void bcast_beta_k(float* brow, const float* __restrict__ bsh, int64_t nnz, int m, int d) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nnz * m) return;
  const int64_t t = i / m;
  const int k = (int)(i - t * m);
  brow[i] = bsh[t * 2 + (k >= d ? 1 : 0)];
}

// shared gradient of side s of subdomain b = sum over the side's rows of
// w[row] x the row's gradient (one block per (b, side))
__global__ void reduce_alpha_k(float* gash, const float* __restrict__ garow, const float* __restrict__ w, Batch bt,
                               int d) {
  const int b = blockIdx.x, side = blockIdx.y;
  const int uc = bt.ucount[b];
  float* dst = gash + bt.aoff[b] / d + side * uc;
  const int r0 = b * bt.m + side * d;
  for (int c = threadIdx.x; c < uc; c += blockDim.x) {
    float s = 0.f;
    for (int k = 0; k < d; ++k) {
      const float wk = w[r0 + k];
      if (wk != 0.f) s = fmaf(wk, garow[bt.rbase[r0 + k] + c], s);
    }
    dst[c] = s;
  }
}

__global__ void reduce_beta_k(float* gbsh, const float* __restrict__ gbrow, const float* __restrict__ w, Batch bt,
                              int d) {
  const int b = blockIdx.x;
  const int64_t s0 = bt.sptr[b], s1 = bt.sptr[b + 1];
  for (int64_t q = s0 * 2 + threadIdx.x; q < s1 * 2; q += blockDim.x) {
    const int64_t t = q >> 1;
    const int side = (int)(q & 1);
    const int r0 = b * bt.m + side * d;
    float s = 0.f;
    for (int k = 0; k < d; ++k) {
      const float wk = w[r0 + k];
      if (wk != 0.f) s = fmaf(wk, gbrow[t * bt.m + side * d + k], s);
    }
    gbsh[q] = s;
  }
}

// d(sum_rows w g)/dl and /du at the currently unstable neurons of columns
// [col0, nd_x) of handle X, added into dL, dU [B][nd].  A row uses the upper
// chord u (z - l)/(u - l) where its stored A is negative; with zbar the
// adjoint's pre-activation there, the chord term A (s zbar - s l) has
// d/dl = A u (zbar - u)/(u - l)^2 and d/du = A l (l - zbar)/(u - l)^2.
__global__ void cot_k(float* dL, float* dU, const uint32_t* __restrict__ status, const float* __restrict__ acomp,
                      const float* __restrict__ zchord, const float* __restrict__ w, const float* __restrict__ lcur,
                      const float* __restrict__ ucur, Batch bt, int col0, int nd_x, int nd, int B) {
  const int ncol = nd_x - col0;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (ncol <= 0 || i >= (int64_t)B * ncol) return;
  const int b = (int)(i / ncol);
  const int c = col0 + (int)(i - (int64_t)b * ncol);
  const uint32_t rec = status[(int64_t)b * nd_x + c];
  if ((rec & kKindMask) != kUnstable) return;
  const int64_t cb = (int64_t)b * nd + c;
  const float l = lcur[cb], u = ucur[cb];
  const float den = u - l;
  const float inv2 = 1.f / (den * den);
  const uint32_t cidx = rec & kCidxMask;
  float dl = 0.f, du = 0.f;
  for (int k = 0; k < bt.m; ++k) {
    const int r = b * bt.m + k;
    const float wk = w ? w[r] : 1.f;
    if (wk == 0.f) continue;
    const int64_t ai = bt.rbase[r] + cidx;
    const float a = acomp[ai];
    if (!(a < 0.f)) continue;
    const float z = zchord[ai];
    dl = fmaf(wk * a, u * (z - u), dl);
    du = fmaf(wk * a, l * (l - z), du);
  }
  dL[cb] += dl * inv2;
  dU[cb] += du * inv2;
}

// row weights of the pass of layer (off, d): the bound cotangents where the
// computed bound is the one in use (lower rows: dL; upper rows: -dU, their
// bound being -u)
__global__ void weights_k(float* w, const float* __restrict__ dL, const float* __restrict__ dU,
                          const uint8_t* __restrict__ ml, const uint8_t* __restrict__ mu, int B, int d, int off,
                          int nd) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)B * d) return;
  const int b = (int)(i / d);
  const int j = (int)(i - (int64_t)b * d);
  const int64_t c = (int64_t)b * nd + off + j;
  w[(int64_t)b * 2 * d + j] = ml[c] ? dL[c] : 0.f;
  w[(int64_t)b * 2 * d + d + j] = mu[c] ? -dU[c] : 0.f;
}

// shared alpha' at CROWN's adaptive slope of the root bounds: block (b, side)
// fills its uc_b entries from the default-slope table adef [B][nd_x] through
// b's unstable list
__global__ void alpha_init_k(float* ash, const int* __restrict__ ulist, const int64_t* __restrict__ uoff, Batch bt,
                             int d) {
  const int b = blockIdx.x, side = blockIdx.y;
  const int uc = bt.ucount[b];
  float* dst = ash + bt.aoff[b] / d + side * uc;
  const int* src = ulist + uoff[b];
  const float* ad = bt.adef + (int64_t)b * bt.nd;
  for (int c = threadIdx.x; c < uc; c += blockDim.x) dst[c] = ad[src[c]];
}

}  // namespace

void launch_joint_alpha_init(float* ash, const int* ulist, const int64_t* uoff, const Batch& bt, int B, int d,
                             hipStream_t s) {
  if (B > 0) alpha_init_k<<<dim3(B, 2), 256, 0, s>>>(ash, ulist, uoff, bt, d);
}

void launch_joint_refresh(uint32_t* status, const uint32_t* status0, float2* chord, const float* lcur,
                          const float* ucur, int B, int nd_x, int nd, hipStream_t s) {
  const int64_t n = (int64_t)B * nd_x;
  if (n > 0) refresh_k<<<nblk(n, 256), 256, 0, s>>>(status, status0, chord, lcur, ucur, B, nd_x, nd);
}

void launch_joint_clip(const float* lb, int d, int off, const float* lroot, const float* uroot, float* lcur,
                       float* ucur, uint8_t* ml, uint8_t* mu, int B, int nd, hipStream_t s) {
  const int64_t n = (int64_t)B * d;
  if (n > 0) clip_k<<<nblk(n, 256), 256, 0, s>>>(lb, d, off, lroot, uroot, lcur, ucur, ml, mu, B, nd);
}

void launch_joint_bcast(float* arow, const float* ash, float* brow, const float* bsh, const Batch& bt, int d,
                        int64_t nnz, hipStream_t s) {
  if (bt.n_rows > 0) bcast_alpha_k<<<bt.n_rows, 256, 0, s>>>(arow, ash, bt, d);
  if (nnz > 0) bcast_beta_k<<<nblk(nnz * bt.m, 256), 256, 0, s>>>(brow, bsh, nnz, bt.m, d);
}

void launch_joint_reduce(float* gash, const float* garow, float* gbsh, const float* gbrow, const float* w,
                         const Batch& bt, int B, int d, int64_t nnz, hipStream_t s) {
  if (B <= 0) return;
  reduce_alpha_k<<<dim3(B, 2), 256, 0, s>>>(gash, garow, w, bt, d);
  if (nnz > 0) reduce_beta_k<<<B, 256, 0, s>>>(gbsh, gbrow, w, bt, d);
}

void launch_joint_cot(float* dL, float* dU, const uint32_t* status, const float* acomp, const float* zchord,
                      const float* w, const float* lcur, const float* ucur, const Batch& bt, int col0, int nd_x,
                      int nd, int B, hipStream_t s) {
  const int64_t n = (int64_t)B * (nd_x - col0);
  if (n > 0)
    cot_k<<<nblk(n, 256), 256, 0, s>>>(dL, dU, status, acomp, zchord, w, lcur, ucur, bt, col0, nd_x, nd, B);
}

void launch_joint_weights(float* w, const float* dL, const float* dU, const uint8_t* ml, const uint8_t* mu, int B,
                          int d, int off, int nd, hipStream_t s) {
  const int64_t n = (int64_t)B * d;
  if (n > 0) weights_k<<<nblk(n, 256), 256, 0, s>>>(w, dL, dU, ml, mu, B, d, off, nd);
}

}  // namespace cvb
