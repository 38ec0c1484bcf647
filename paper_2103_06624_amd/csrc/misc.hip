// Small kernels of libcvbound: set-up (relaxation chords, subdomain status,
// specification merge), the top ReLU layer, bound assembly and projected Adam.
#include "common.h"
#include "internal.h"

namespace cvb {

namespace {

__global__ void prep_chord_k(const float* __restrict__ l, const float* __restrict__ u, float2* chord, float* adef,
                             int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float lo = l[i], up = u[i];
  float2 c = make_float2(0.f, 0.f);
  if (lo < 0.f && up > 0.f) {
    // upper chord of ReLU on [l, u]: zhat <= u/(u-l) (z - l)  (Lemma 2.1)
    const float den = up - lo;
    c.x = up / den;
    c.y = -up * lo / den;
  }
  chord[i] = c;
  adef[i] = (up >= -lo) ? 1.f : 0.f;  // CROWN's adaptive lower slope
}

__global__ void status_fill_k(uint32_t* status, const uint32_t* __restrict__ root_kind, const int* __restrict__ prop,
                              int B, int nd) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)B * nd) return;
  const int b = (int)(i / nd);
  const int j = (int)(i - (int64_t)b * nd);
  status[i] = root_kind[(int64_t)prop[b] * nd + j];
}

__global__ void status_split_k(uint32_t* status, const int* __restrict__ split_dom, const int* __restrict__ split_col,
                               const int8_t* __restrict__ side, int64_t nnz, int nd) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nnz) return;
  const int b = split_dom[s];
  status[(int64_t)b * nd + split_col[s]] = kSplit | (side[s] > 0 ? kSidePos : 0u) | (uint32_t)s;
}

// A(L-1) = C_p W(L) and c = C_p b(L) for every property and spec row
// (the specification merged into the last layer, Sec. 2.1).
__global__ void spec_merge_k(const float* __restrict__ C, const float* __restrict__ W, int ldw,
                             const float* __restrict__ b, int m, int dL, int dprev, float* CW, int ldcw, float* Cb) {
  const int pk = blockIdx.x;  // p * m + k
  const float* c = C + (int64_t)pk * dL;
  for (int j = threadIdx.x; j < dprev; j += blockDim.x) {
    float s = 0.f;
    for (int o = 0; o < dL; ++o) s = fmaf(c[o], W[(int64_t)o * ldw + j], s);
    CW[(int64_t)pk * ldcw + j] = s;
  }
  if (threadIdx.x == 0) {
    float s = 0.f;
    for (int o = 0; o < dL; ++o) s = fmaf(c[o], b[o], s);
    Cb[pk] = s;
  }
}

// Specification [I; -I] on layer i (row k < d: +e_k, else -e_{k-d}): A = +-W(i) row.
__global__ void spec_identity_k(const float* __restrict__ Wd, int ldw, const float* __restrict__ wc, ConvGeom g,
                                int use_conv, const float* __restrict__ bias_full, int d, int dprev, float* CW,
                                int ldcw, float* Cb) {
  const int k = blockIdx.x;
  const int o = k < d ? k : k - d;
  const float sg = k < d ? 1.f : -1.f;
  float* out = CW + (int64_t)k * ldcw;
  if (!use_conv) {
    for (int j = threadIdx.x; j < dprev; j += blockDim.x) out[j] = sg * Wd[(int64_t)o * ldw + j];
  } else {
    const int pos = g.ho * g.wo;
    const int co = o / pos, q = o - co * pos;
    const int oy = q / g.wo, ox = q - oy * g.wo;
    for (int j = threadIdx.x; j < dprev; j += blockDim.x) {
      const int ci = j / (g.hi * g.wi), r = j - ci * g.hi * g.wi;
      const int iy = r / g.wi, ix = r - iy * g.wi;
      const int ky = iy - oy * g.s + g.p, kx = ix - ox * g.s + g.p;
      float val = 0.f;
      if (ky >= 0 && ky < g.k && kx >= 0 && kx < g.k) val = wc[(((int64_t)co * g.ci + ci) * g.k + ky) * g.k + kx];
      out[j] = sg * val;
    }
  }
  if (threadIdx.x == 0) Cb[k] = sg * bias_full[o];
}

// The top ReLU layer: relax A(L-1) = C_p W(L) row by row (or concretise it
// directly when the network has no ReLU layer).  One wave per row; each lane
// takes E neurons at a time and issues their loads together (row operand,
// status, bias, then the chord and variable that depend on the status).
__global__ __launch_bounds__(256) void top_k(TopArgs a) {
  constexpr int E = 4;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= a.bt.n_rows) return;
  const RowInfo ri = row_info(a.bt, row);
  const float* cw = a.CW + ri.p * a.cw_pstride + (int64_t)ri.k * a.ldcw;
  const uint32_t* st = a.bt.status + (int64_t)ri.b * a.bt.nd + a.e.layer_off;
  float cst = 0.f, cer = 0.f;
  for (int j0 = lane; j0 < a.n; j0 += 64 * E) {
    float av[E], b1[E], b2[E];
    uint32_t rec[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int j = j0 + 64 * e;
      const bool ok = j < a.n;
      av[e] = ok ? cw[j] : 0.f;
      rec[e] = kInactive;
      b1[e] = 0.f;
      b2[e] = 0.f;
      if (a.conc) {
        const int64_t pb = (int64_t)ri.p * a.bt.d0 + j;
        if (ok && a.bt.l2x0) {
          b1[e] = a.bt.l2x0[pb];
        } else if (ok) {
          b1[e] = a.bt.xlo[pb];
          b2[e] = a.bt.xhi[pb];
        }
      } else if (ok) {
        rec[e] = st[j];
        b1[e] = a.e.bias[j];
      }
    }
    if (a.conc) {
#pragma unroll
      for (int e = 0; e < E; ++e)
        if (j0 + 64 * e < a.n) {
          if (a.bt.l2x0) {  // l_p ball: A x0 here, - eps ||A||_q in the final sum
            cst = fmaf(av[e], b1[e], cst);
            lp_entry(av[e], a.bt.lpq, &cer);
          } else {
            const float tm = conc_term(av[e], b1[e], b2[e]);
            cst += tm;
            cer = fmaf(a.bt.sg, fabsf(tm), cer);
          }
        }
      continue;
    }
    float2 ch[E];
    float al[E], be[E], sw[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int j = j0 + 64 * e;
      const int64_t pc = (int64_t)ri.p * a.bt.nd + a.e.layer_off + j;
      ch[e] = (rec[e] & kKindMask) == kUnstable ? a.bt.chord[pc] : make_float2(0.f, 0.f);
      relax_vars(a.bt, a.v, ri, rec[e], pc, &al[e], &be[e]);
      sw[e] = a.bt.sw && j < a.n ? a.bt.sw[pc] : 0.f;
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int j = j0 + 64 * e;
      if (j >= a.n) continue;
      if (a.v.acomp && (rec[e] & kKindMask) == kUnstable) a.v.acomp[ri.abase + (rec[e] & kCidxMask)] = av[e];
      const float lam =
          relax_value(a.bt, a.v, ri, rec[e], ch[e], relax_pick(rec[e], al[e], be[e]), av[e], b1[e], &cst);
      a.e.out[(int64_t)row * a.e.ldo + j] = lam;
      cer = fmaf(fabsf(lam), sw[e], cer);
    }
  }
  cst = wave_sum(cst);
  if (lane == 0) a.e.part[(int64_t)a.e.slot0 * a.bt.n_rows + row] = cst + a.Cb[ri.p * a.cb_pstride + ri.k];
  if (a.e.perr || a.e.psq) {
    // cer: the rounding-error bound, or over an l_p ball with no ReLU layer
    // the sum of |A|^q (then the error slot keeps only the specification's
    // error)
    const bool sq = a.conc && a.bt.l2x0;
    cer = wave_sum(cer);
    if (lane == 0) {
      const int64_t at = (int64_t)a.e.slot0 * a.bt.n_rows + row;
      if (a.e.perr) a.e.perr[at] = (sq ? 0.f : cer) + (a.err0 ? a.err0[ri.p * a.bt.m + ri.k] : 0.f);
      if (a.e.psq) a.e.psq[at] = sq ? cer : 0.f;
    }
  }
}

// ub = C_p W(L) zhat(L-1) + C_p b(L) for each row: the network's output at
// x* under the row's specification row (one wave per row).
__global__ __launch_bounds__(256) void top_dot_k(TopArgs a, const float* __restrict__ z, int ldz, float* ub) {
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= a.bt.n_rows) return;
  const RowInfo ri = row_info(a.bt, row);
  const float* cw = a.CW + ri.p * a.cw_pstride + (int64_t)ri.k * a.ldcw;
  const float* zr = z + (int64_t)row * ldz;
  float s = 0.f;
  for (int j = lane; j < a.n; j += 64) s = fmaf(cw[j], zr[j], s);
  s = wave_sum(s);
  if (lane == 0) ub[row] = s + a.Cb[ri.p * a.cb_pstride + ri.k];
}

__global__ __launch_bounds__(256) void fill_i32_k(int* p, int v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = v;
}

// lb = sum of the partial constants of a row, in a fixed order
// (deterministic).  Partials are slot-major [slot][row].  Wave g of a block
// sums slots g, g+4, g+8, ... of 64 rows with 8 loads in flight per lane; the
// four sums are then added in wave order.
// Sound mode (perr set): the rounding-error partials are summed the same way,
// scaled by `scale` for their own rounding, and the bound is lowered by them,
// each step rounded outward.  l_p ball (psq set): the partial sums of
// |A(0)|^q give ||A(0)||_q and the bound is lowered by eps_p ||A(0)||_q (in
// sound mode, l2 only, by an upper bound on it, plus the concretisation sum's
// own rounding); l2s[row] receives eps_p / ||A(0)||_q^(q-1) (0 when A(0) = 0),
// the scale of the adjoint's x* = x0 - l2s sign(A(0)) |A(0)|^(q-1).
__device__ __forceinline__ float slot_sum(const float* __restrict__ part, int n_used, int n_rows, int r, int g) {
  float s = 0.f;
  int t = g;
  for (; t + 28 < n_used; t += 32) {
    float x[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) x[q] = part[(int64_t)(t + 4 * q) * n_rows + r];
#pragma unroll
    for (int q = 0; q < 8; ++q) s += x[q];
  }
  for (; t < n_used; t += 4) s += part[(int64_t)t * n_rows + r];
  return s;
}

__global__ __launch_bounds__(256) void finalize_k(const float* __restrict__ part, const float* __restrict__ perr,
                                                  float scale, const float* __restrict__ psq, L2Final l2,
                                                  int n_used, int n_rows, float* lb, float* best, int first,
                                                  int* improved) {
  __shared__ float red[4][64], rede[4][64], redq[4][64];
  const int rl = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int r = blockIdx.x * 64 + rl;
  red[g][rl] = r < n_rows ? slot_sum(part, n_used, n_rows, r, g) : 0.f;
  if (perr) rede[g][rl] = r < n_rows ? slot_sum(perr, n_used, n_rows, r, g) : 0.f;
  if (psq) redq[g][rl] = r < n_rows ? slot_sum(psq, n_used, n_rows, r, g) : 0.f;
  __syncthreads();
  if (g == 0 && r < n_rows) {
    float tot = ((red[0][rl] + red[1][rl]) + red[2][rl]) + red[3][rl];
    float err = 0.f;
    if (perr) err = nextafterf((((rede[0][rl] + rede[1][rl]) + rede[2][rl]) + rede[3][rl]) * scale, INFINITY);
    if (psq) {
      const int p = l2.prop[r / l2.m];
      const float sq = ((redq[0][rl] + redq[1][rl]) + redq[2][rl]) + redq[3][rl];
      const float eps = l2.eps[p];
      float nrm;
      if (l2.q == 2.f) {
        nrm = sqrtf(sq);
        if (l2.l2s) l2.l2s[r] = nrm > 0.f ? eps / nrm : 0.f;
      } else {
        // ||A||_q = S^(1/q); the adjoint's scale eps / ||A||_q^(q-1) = eps ||A||_q / S
        nrm = sq > 0.f ? exp2f(log2f(sq) / l2.q) : 0.f;
        if (l2.l2s) l2.l2s[r] = sq > 0.f ? eps * (nrm / sq) : 0.f;
      }
      if (perr) {
        // sound: ||A(0)||_2 <= nrm * fac (the sum of squares and the square
        // root rounded), and the float sum A(0) x0 is off by at most
        // g sum |a x0| <= g ||A(0)||_2 ||x0||_2
        const float nup = nextafterf(nrm * l2.fac, INFINITY);
        const float m2 = nextafterf(nextafterf(eps * nup, INFINITY) + nextafterf(l2.g * nup * l2.x0n[p], INFINITY),
                                    INFINITY);
        err = nextafterf(err + m2, INFINITY);
      } else {
        tot = fmaf(-eps, nrm, tot);
      }
    }
    if (perr) tot = nextafterf(tot - err, -INFINITY);
    if (lb) lb[r] = tot;
    if (best) {
      const bool up = first || tot > best[r];
      if (up) best[r] = tot;
      if (improved) improved[r] = up ? 1 : 0;
    }
  }
}

// The variables of every row whose bound improved (improved[row]): alpha's
// [U_p] block of the row and beta's entries of the row (one per split of its
// subdomain, stride m), copied to abest / bbest.  One block per row.
__global__ __launch_bounds__(256) void keep_best_k(const float* __restrict__ alpha, const float* __restrict__ beta,
                                                   float* abest, float* bbest, const int* __restrict__ improved,
                                                   Batch bt) {
  const int row = blockIdx.x;
  if (!improved[row]) return;
  const RowInfo ri = row_info(bt, row);
  const int U = bt.ucount[ri.p];
  for (int t = threadIdx.x; t < U; t += 256) abest[ri.abase + t] = alpha[ri.abase + t];
  const int64_t s0 = bt.sptr[ri.b], s1 = bt.sptr[ri.b + 1];
  for (int64_t t = s0 + threadIdx.x; t < s1; t += 256) bbest[t * bt.m + ri.k] = beta[t * bt.m + ri.k];
}

// Projected Adam ascent step (Kingma & Ba, beta1 0.9, beta2 0.999, eps 1e-8).
__global__ void adam_k(float* x, const float* __restrict__ g, float* m1, float* m2, int64_t n, float lr, float bc1,
                       float bc2, float lo, float hi) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  adam_apply(x, m1, m2, i, g[i], lr, bc1, bc2, lo, hi);
}

// The steps a conv layer's adjoint left to after the pass (Vars::gsplit):
// for split t of a layer whose columns are flagged in defer and spec row k,
// the Adam step of beta[t, k] on its staged gradient and the zero-gradient
// step of the split neuron's alpha entry in that row -- the fused epilogue's
// steps, in the same arithmetic.
__global__ void split_adam_k(Batch bt, Vars v, const int* __restrict__ split_dom, const int* __restrict__ split_col,
                             const uint8_t* __restrict__ defer, int64_t nnz) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nnz * bt.m) return;
  const int64_t t = i / bt.m;
  const int k = (int)(i - t * bt.m);
  const int col = split_col[t];
  if (!defer[col]) return;
  const int b = split_dom[t];
  const int p = bt.prop[b];
  const int64_t ai = bt.rbase[(int64_t)b * bt.m + k] + bt.cidx[(int64_t)p * bt.nd + col];
  adam_apply(v.beta_w, v.mb, v.vb, i, v.gsplit[i], v.lr_b, v.bc1, v.bc2, 0.f, INFINITY);
  // the alpha entry's zero-gradient step often leaves it and its moments as
  // they were (moments at zero): only what changed is stored (scattered
  // entries, one per row and split)
  const float xv = v.alpha_w[ai], m1v = v.ma[ai], m2v = v.va[ai];
  float m1n, m2n;
  const float xn = adam_values(0.f, v.lr_a, v.bc1, v.bc2, 0.f, 1.f, xv, m1v, m2v, m1n, m2n);
  if (__float_as_uint(m1n) != __float_as_uint(m1v)) v.ma[ai] = m1n;
  if (__float_as_uint(m2n) != __float_as_uint(m2v)) v.va[ai] = m2n;
  if (__float_as_uint(xn) != __float_as_uint(xv)) v.alpha_w[ai] = xn;
}

__global__ void fill_k(float* p, float v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// alpha <- default slope of each entry's neuron; one block per row.  ulist
// holds each property's unstable neurons (nd-axis index), uoff its offsets.
__global__ void alpha_default_k(float* alpha, const int* __restrict__ ulist, const int64_t* __restrict__ uoff,
                                Batch bt) {
  const int row = blockIdx.x;
  const RowInfo ri = row_info(bt, row);
  const int U = bt.ucount[ri.p];
  const int* src = ulist + uoff[ri.p];
  const float* ad = bt.adef + (int64_t)ri.p * bt.nd;
  for (int t = threadIdx.x; t < U; t += blockDim.x) alpha[ri.abase + t] = ad[src[t]];
}

inline unsigned nblk(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

void launch_prep_chord(const float* l, const float* u, float2* chord, float* adef, int64_t n, hipStream_t s) {
  if (n > 0) prep_chord_k<<<nblk(n, 256), 256, 0, s>>>(l, u, chord, adef, n);
}
void launch_status_fill(uint32_t* status, const uint32_t* root_kind, const int* prop, int B, int nd, hipStream_t s) {
  const int64_t n = (int64_t)B * nd;
  if (n > 0) status_fill_k<<<nblk(n, 256), 256, 0, s>>>(status, root_kind, prop, B, nd);
}
void launch_status_split(uint32_t* status, const int* split_dom, const int* split_col, const int8_t* side, int64_t nnz,
                         int nd, hipStream_t s) {
  if (nnz > 0) status_split_k<<<nblk(nnz, 256), 256, 0, s>>>(status, split_dom, split_col, side, nnz, nd);
}
void launch_spec_merge(const float* C, const float* W, int ldw, const float* b, int P, int m, int dL, int dprev,
                       float* CW, int ldcw, float* Cb, hipStream_t s) {
  spec_merge_k<<<P * m, 256, 0, s>>>(C, W, ldw, b, m, dL, dprev, CW, ldcw, Cb);
}
void launch_spec_identity(const float* Wdense, int ldw, const float* wconv, const ConvGeom* g, const float* bias_full,
                          int d, int dprev, float* CW, int ldcw, float* Cb, hipStream_t s) {
  ConvGeom gg = g ? *g : ConvGeom{};
  spec_identity_k<<<2 * d, 256, 0, s>>>(Wdense, ldw, wconv, gg, g ? 1 : 0, bias_full, d, dprev, CW, ldcw, Cb);
}
void launch_top_dot(const TopArgs& a, const float* z, int ldz, float* ub, hipStream_t s) {
  if (a.bt.n_rows > 0) launch_k(top_dot_k, nblk(a.bt.n_rows, 4), 256, 0, s, a, z, ldz, ub);
}

void launch_fill_i32(int* p, int v, int64_t n, hipStream_t s) {
  if (n > 0) fill_i32_k<<<nblk(n, 256), 256, 0, s>>>(p, v, n);
}

void launch_top(const TopArgs& a, hipStream_t s) { launch_k(top_k, nblk(a.bt.n_rows, 4), 256, 0, s, a); }
void launch_finalize(const float* part, const float* perr, float scale, const float* psq, const L2Final& l2,
                     int n_slots, int n_used, int n_rows, float* lb, float* best, int first, hipStream_t s,
                     int* improved) {
  (void)n_slots;
  launch_k(finalize_k, nblk(n_rows, 64), 256, 0, s, part, perr, scale, psq, l2, n_used, n_rows, lb, best, first,
           improved);
}
void launch_keep_best(const float* alpha, const float* beta, float* abest, float* bbest, const int* improved,
                      const Batch& bt, hipStream_t s) {
  if (bt.n_rows > 0) launch_k(keep_best_k, (unsigned)bt.n_rows, 256, 0, s, alpha, beta, abest, bbest, improved, bt);
}
void launch_split_adam(const Batch& bt, const Vars& v, const int* split_dom, const int* split_col,
                       const uint8_t* defer, int64_t nnz, hipStream_t s) {
  const int64_t n = nnz * bt.m;
  if (n <= 0) return;
  split_adam_k<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(bt, v, split_dom, split_col, defer, nnz);
}

void launch_adam(float* x, const float* g, float* m1, float* m2, int64_t n, float lr, float bc1, float bc2, float lo,
                 float hi, hipStream_t s) {
  if (n > 0) adam_k<<<nblk(n, 256), 256, 0, s>>>(x, g, m1, m2, n, lr, bc1, bc2, lo, hi);
}
void launch_fill(float* p, float v, int64_t n, hipStream_t s) {
  if (n > 0) fill_k<<<nblk(n, 256), 256, 0, s>>>(p, v, n);
}
void launch_alpha_default(float* alpha, const int* ulist, const int64_t* uoff, const Batch& bt, hipStream_t s) {
  if (bt.n_rows > 0) alpha_default_k<<<bt.n_rows, 256, 0, s>>>(alpha, ulist, uoff, bt);
}

}  // namespace cvb
