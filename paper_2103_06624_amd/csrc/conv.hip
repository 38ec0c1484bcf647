// Back-substitution through convolution layers and the adjoint's forward
// convolution (gfx950).
//
// Back-substitution A(i-1) = Lambda(i) W(i) through a conv layer is the
// transposed convolution of each row of Lambda(i) with the layer's kernel.
// It is computed as an implicit GEMM per output position: for an output
// (c_in, y, x) the K dimension runs over (c_out, valid taps), where for
// stride s the valid taps are those with ky = (y + pad) mod s (+ s, ...), so
// the positions are processed in stride-parity classes and every lane of a
// wave shares the same taps and the same weights.  Each thread keeps all
// C_in outputs of one position in registers, so an LDS read of Lambda feeds
// C_in FMAs.  The adjoint's forward conv keeps all C_out outputs of one
// position in registers likewise.
#include "common.h"
#include "internal.h"

namespace cvb {

namespace {

// Row slice of the block: RB rows per block, positions per row `pos`, 256 threads.
struct Slice {
  int rb;     // rows per block
  int row0;   // first row of the block
  int rl;     // this thread's row (local)
  int q0;     // this thread's first position
  int qstep;  // position stride
};

__device__ __forceinline__ Slice slice_of(int pos) {
  Slice s;
  s.rb = pos >= 256 ? 1 : 256 / pos;
  s.row0 = blockIdx.x * s.rb;
  if (s.rb == 1) {
    s.rl = 0;
    s.q0 = threadIdx.x;
    s.qstep = 256;
  } else {
    s.rl = threadIdx.x / pos;
    s.q0 = threadIdx.x - s.rl * pos;
    s.qstep = pos;
  }
  return s;
}

// Sum `x` over the threads of each local row and return the total to thread 0
// of that row (rows own whole waves since pos is a multiple of 64).
__device__ __forceinline__ float row_sum(float x, int pos, float* red) {
  x = wave_sum(x);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) red[w] = x;
  __syncthreads();
  float s = 0.f;
  const int wpr = pos >= 256 ? 4 : pos / 64;  // waves per row
  if (threadIdx.x < 4 && threadIdx.x < 256 / (wpr * 64)) {
    for (int t = 0; t < wpr; ++t) s += red[threadIdx.x * wpr + t];
  }
  return s;
}

template <int CI, int MODE>
__global__ __launch_bounds__(256) void convt_bwd(const float* __restrict__ lam, int ldl, const float* __restrict__ w,
                                                 ConvGeom g, int M, int uniform, Batch bt, Vars v, Epi e) {
  extern __shared__ float smem[];
  __shared__ float red[4], rede[4];
  const int pos = g.hi * g.wi;             // positions of the output plane
  const int din = g.co * g.ho * g.wo;      // length of a Lambda row
  const Slice sl = slice_of(pos);
  float* lrow = smem;                                   // [rb][din]
  const int w32 = bt.w64 * 2;
  uint32_t* bits_all = reinterpret_cast<uint32_t*>(smem + sl.rb * din);  // [rb][2][w32] (conc mode)
  for (int t = threadIdx.x; t < sl.rb * din; t += 256) {
    const int rr = t / din, jj = t - rr * din;
    const int row = sl.row0 + rr;
    lrow[t] = row < M ? lam[(int64_t)row * ldl + jj] : 0.f;
  }
  if (MODE == kBwdConc && v.xpos)
    for (int t = threadIdx.x; t < sl.rb * 2 * w32; t += 256) bits_all[t] = 0u;
  __syncthreads();
  uint32_t* bits = bits_all + sl.rl * 2 * w32;

  const int row = sl.row0 + sl.rl;
  const bool rok = row < M;
  RowInfo ri;
  if (rok) ri = row_info(bt, row);
  const float* L = lrow + sl.rl * din;
  const int s = g.s, k = g.k, pad = g.p;
  const int hs = g.hi / s, ws = g.wi / s, cls_n = hs * ws;
  float cst = 0.f, cer = 0.f;
  for (int q = sl.q0; q < pos; q += sl.qstep) {
    // position q in parity-class order
    int cls = q / cls_n;
    const int e0 = q - cls * cls_n;
    const int yy = e0 / ws, xx = e0 - yy * ws;
    if (uniform) cls = __builtin_amdgcn_readfirstlane(cls);
    const int py = cls / s, px = cls - (cls / s) * s;
    const int y = yy * s + py, x = xx * s + px;
    const int ky0 = (py + pad) % s, kx0 = (px + pad) % s;
    float acc[CI];
#pragma unroll
    for (int c = 0; c < CI; ++c) acc[c] = 0.f;
    for (int co = 0; co < g.co; ++co) {
      for (int ky = ky0; ky < k; ky += s) {
        const int oy = (y + pad - ky) / s;
        if (oy < 0 || oy >= g.ho) continue;
        for (int kx = kx0; kx < k; kx += s) {
          const int ox = (x + pad - kx) / s;
          if (ox < 0 || ox >= g.wo) continue;
          const float val = L[(co * g.ho + oy) * g.wo + ox];
          const float* wp = w + ((int64_t)co * CI * k + ky) * k + kx;
#pragma unroll
          for (int c = 0; c < CI; ++c) acc[c] = fmaf(val, wp[(int64_t)c * k * k], acc[c]);
        }
      }
    }
    if (!rok) continue;
#pragma unroll
    for (int c = 0; c < CI; ++c) {
      const int j = c * pos + y * g.wi + x;
      const float a = acc[c];
      if (MODE == kBwdRelax) {
        e.out[(int64_t)row * e.ldo + j] = relax_bwd(bt, v, ri, e.layer_off, j, a, e.bias[j], &cst, &cer);
      } else if (bt.l2x0) {  // l2 ball: A(0) x0 here, - eps ||A(0)||_2 in the final sum
        const int64_t pb = (int64_t)ri.p * bt.d0 + j;
        cst = fmaf(a, bt.l2x0[pb], cst);
        cer = fmaf(a, a, cer);
        if (v.xdense) v.xdense[(int64_t)row * v.ldx + j] = a;  // A(0) itself for the adjoint
      } else {
        const int64_t pb = (int64_t)ri.p * bt.d0 + j;
        const float tm = conc_term(a, bt.xlo[pb], bt.xhi[pb]);
        cst += tm;
        cer = fmaf(bt.sg, fabsf(tm), cer);
        if (v.xpos) {
          if (a > 0.f) atomicOr(&bits[j >> 5], 1u << (j & 31));
          if (a < 0.f) atomicOr(&bits[w32 + (j >> 5)], 1u << (j & 31));
        }
      }
    }
  }
  const float tot = row_sum(cst, pos, red);
  if (threadIdx.x < sl.rb) {
    const int r2 = sl.row0 + threadIdx.x;
    if (r2 < M) e.part[(int64_t)e.slot0 * M + r2] = tot;
  }
  float* const p2 = e.perr ? e.perr : e.psq;  // rounding-error bound, or the sum of A(0)^2 (l2 ball)
  if (p2) {
    const float ter = row_sum(cer, pos, rede);
    if (threadIdx.x < sl.rb) {
      const int r2 = sl.row0 + threadIdx.x;
      if (r2 < M) p2[(int64_t)e.slot0 * M + r2] = ter;
    }
  }
  if (MODE == kBwdConc && v.xpos) {
    __syncthreads();
    for (int t = threadIdx.x; t < sl.rb * w32; t += 256) {
      const int rr = t / w32, wd = t - rr * w32;
      const int r2 = sl.row0 + rr;
      if (r2 < M) {
        reinterpret_cast<uint32_t*>(v.xpos + (int64_t)r2 * bt.w64)[wd] = bits_all[rr * 2 * w32 + wd];
        reinterpret_cast<uint32_t*>(v.xneg + (int64_t)r2 * bt.w64)[wd] = bits_all[rr * 2 * w32 + w32 + wd];
      }
    }
  }
}

template <int CO, int MODE>
__global__ __launch_bounds__(256) void conv_fwd(const float* __restrict__ zin, int ldi, const float* __restrict__ w,
                                                ConvGeom g, int M, int last, Batch bt, Vars v, Epi e) {
  extern __shared__ float smem[];
  const int pos = g.ho * g.wo;
  const int din = g.ci * g.hi * g.wi;
  const Slice sl = slice_of(pos);
  for (int t = threadIdx.x; t < sl.rb * din; t += 256) {
    const int rr = t / din, jj = t - rr * din;
    const int row = sl.row0 + rr;
    float val = 0.f;
    if (row < M) {
      if (MODE == kFwdX) {
        const int p = bt.prop[row / bt.m];
        const uint64_t wp = v.xpos[(int64_t)row * bt.w64 + (jj >> 6)];
        const uint64_t wn = v.xneg[(int64_t)row * bt.w64 + (jj >> 6)];
        const int64_t pb = (int64_t)p * bt.d0 + jj;
        val = xstar((wp >> (jj & 63)) & 1, (wn >> (jj & 63)) & 1, bt.xlo[pb], bt.xhi[pb]);
      } else {
        val = zin[(int64_t)row * ldi + jj];
      }
    }
    smem[t] = val;
  }
  __syncthreads();
  const int row = sl.row0 + sl.rl;
  if (row >= M) return;
  const RowInfo ri = row_info(bt, row);
  const float* Z = smem + sl.rl * din;
  const int s = g.s, k = g.k, pad = g.p;
  for (int q = sl.q0; q < pos; q += sl.qstep) {
    const int oy = q / g.wo, ox = q - oy * g.wo;
    float acc[CO];
#pragma unroll
    for (int c = 0; c < CO; ++c) acc[c] = 0.f;
    for (int ci = 0; ci < g.ci; ++ci) {
      for (int ky = 0; ky < k; ++ky) {
        const int iy = oy * s - pad + ky;
        if (iy < 0 || iy >= g.hi) continue;
        for (int kx = 0; kx < k; ++kx) {
          const int ix = ox * s - pad + kx;
          if (ix < 0 || ix >= g.wi) continue;
          const float val = Z[(ci * g.hi + iy) * g.wi + ix];
          const float* wp = w + ((int64_t)ci * k + ky) * k + kx;
#pragma unroll
          for (int c = 0; c < CO; ++c) acc[c] = fmaf(val, wp[(int64_t)c * g.ci * k * k], acc[c]);
        }
      }
    }
#pragma unroll
    for (int c = 0; c < CO; ++c) {
      const int j = c * pos + q;
      // l2 ball, first layer: W(1) x* + b(1) = (W(1) x0 + b(1)) - l2s (W(1) A(0))
      const float zb = e.wx0 ? fmaf(-v.l2s[row], acc[c], e.wx0[(int64_t)ri.p * e.n + j]) : acc[c] + e.bias[j];
      if (v.sat) {  // the network itself at x*: every layer's output is kept
        const uint32_t rec = bt.status[(int64_t)ri.b * bt.nd + e.layer_off + j];
        e.out[(int64_t)row * e.ldo + j] = true_relu(rec, zb, v.sat + row);
        continue;
      }
      const float zh = relax_fwd(bt, v, ri, e.layer_off, j, zb);
      if (!last) e.out[(int64_t)row * e.ldo + j] = zh;
    }
  }
}

template <int MODE>
int convt_dispatch(const ConvArgs& a, hipStream_t st) {
  const int pos = a.g.hi * a.g.wi;
  const int rb = pos >= 256 ? 1 : 256 / pos;
  const int din = a.g.co * a.g.ho * a.g.wo;
  size_t sm = (size_t)rb * din * sizeof(float);
  if (MODE == kBwdConc) sm += (size_t)rb * 4 * a.bt.w64 * sizeof(uint32_t);
  const dim3 grid((a.M + rb - 1) / rb), block(256);
#define CVB_CT(CI)                                                                                         \
  case CI:                                                                                                 \
    launch_k(convt_bwd<CI, MODE>, grid, block, sm, st, a.in, a.ldi, a.w, a.g, a.M, a.uniform, a.bt, a.v, a.e); \
    return 0;
  switch (a.g.ci) {
    CVB_CT(1) CVB_CT(2) CVB_CT(3) CVB_CT(4) CVB_CT(8) CVB_CT(16) CVB_CT(32)
    default:
      return -1;
  }
#undef CVB_CT
}

template <int MODE>
int conv_dispatch(const ConvArgs& a, hipStream_t st) {
  const int pos = a.g.ho * a.g.wo;
  const int rb = pos >= 256 ? 1 : 256 / pos;
  const int din = a.g.ci * a.g.hi * a.g.wi;
  const size_t sm = (size_t)rb * din * sizeof(float);
  const dim3 grid((a.M + rb - 1) / rb), block(256);
#define CVB_CF(CO)                                                                                      \
  case CO:                                                                                              \
    launch_k(conv_fwd<CO, MODE>, grid, block, sm, st, a.in, a.ldi, a.w, a.g, a.M, a.last, a.bt, a.v, a.e); \
    return 0;
  switch (a.g.co) {
    CVB_CF(1) CVB_CF(2) CVB_CF(3) CVB_CF(4) CVB_CF(8) CVB_CF(16) CVB_CF(32)
    default:
      return -1;
  }
#undef CVB_CF
}

}  // namespace

bool conv_channels_supported(int c) { return c == 1 || c == 2 || c == 3 || c == 4 || c == 8 || c == 16 || c == 32; }

size_t convt_smem_bytes(const ConvGeom& g, int w64, bool conc) {
  const int pos = g.hi * g.wi;
  const int rb = pos >= 256 ? 1 : 256 / pos;
  return (size_t)rb * g.co * g.ho * g.wo * sizeof(float) + (conc ? (size_t)rb * 4 * w64 * sizeof(uint32_t) : 0);
}

size_t conv_smem_bytes(const ConvGeom& g) {
  const int pos = g.ho * g.wo;
  const int rb = pos >= 256 ? 1 : 256 / pos;
  return (size_t)rb * g.ci * g.hi * g.wi * sizeof(float);
}

int launch_convt_bwd(int mode, const ConvArgs& a, hipStream_t s) {
  return mode == kBwdConc ? convt_dispatch<kBwdConc>(a, s) : convt_dispatch<kBwdRelax>(a, s);
}

int launch_conv_fwd(int mode, const ConvArgs& a, hipStream_t s) {
  return mode == kFwdX ? conv_dispatch<kFwdX>(a, s) : conv_dispatch<kFwd>(a, s);
}

}  // namespace cvb
