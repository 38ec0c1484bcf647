/*
 * cvbound: batched beta-CROWN bound propagation on one MI355X (gfx950).
 *
 * The library computes, for a batch of branch-and-bound subdomains, the
 * beta-CROWN lower bound of each row of C f(x) over an input box (Wang et al.,
 * "Beta-CROWN", NeurIPS 2021, Theorem 3.1 with the recursive form of
 * Eq. definition_A), its gradient with respect to the per-subdomain
 * variables alpha and beta, and a projected-Adam ascent on them
 * (Eq. opt_alpha_beta; 20 Adam iterations with a 0.98 learning-rate decay in
 * the paper's setup, App. C.1).
 *
 * Notation (Sec. 2.1): layer i computes z(i) = W(i) zhat(i-1) + b(i) and
 * zhat(i) = ReLU(z(i)) for i = 1..L-1; layer L is linear; zhat(0) = x.
 * l(i) <= z(i) <= u(i) are intermediate bounds.  A subdomain adds split
 * constraints z(i)_j >= 0 (set Z+) or z(i)_j < 0 (set Z-) (Sec. 2.3).
 *
 * Conventions for every entry point:
 *   - return value 0 on success, a negative CV_E* code on failure; on
 *     failure cv_last_error() gives a message (thread-local), and no output
 *     has been written;
 *   - `stream` is a hipStream_t (NULL = the null stream);
 *   - "host" pointers are read during the call and may be freed afterwards;
 *     "device" pointers are caller-owned device memory, accessed in stream
 *     order after the call returns (asynchronous), float32 and contiguous;
 *   - a handle is not thread-safe: one thread, one stream at a time.
 *
 * Variable layouts (device, float32):
 *   alpha:  for subdomain b with property p, an [m, U_p] block, where U_p is
 *           the number of root-unstable neurons (l < 0 < u) of property p,
 *           listed layer by layer in neuron order; blocks concatenated in
 *           subdomain order (cv_bound_sizes gives the total,
 *           cv_bound_alpha_offset one entry).  Entries of neurons that the
 *           subdomain splits are ignored (gradient 0).
 *   beta:   [nnz, m] in CSR split order (one multiplier per split per spec
 *           row).
 *   bounds: [B, m].
 */
#ifndef CVBOUND_H
#define CVBOUND_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  CV_OK = 0,
  CV_EINVAL = -1,  /* null pointer, bad count or non-finite input           */
  CV_ESHAPE = -2,  /* layer shapes do not chain or are unsupported           */
  CV_ESPLIT = -3,  /* invalid split set (see cv_bound_init)                  */
  CV_ENOMEM = -4,  /* device allocation failed                               */
  CV_EDEVICE = -5  /* a HIP runtime call failed                              */
};

enum { CV_LAYER_DENSE = 0, CV_LAYER_CONV2D = 1 };

/* One affine layer (Sec. 2.1).  Dense: in = (in_c,1,1), out = (out_c,1,1),
 * weight [out_c][in_c] row-major.  Conv2d (cross-correlation, zero padding):
 * weight OIHW [out_c][in_c][k][k], out_h = (in_h + 2 pad - k)/stride + 1.
 * Activations are flattened C,H,W row-major.  bias [out_c].  Host pointers. */
typedef struct cv_layer {
  int32_t type;
  int32_t in_c, in_h, in_w;
  int32_t out_c, out_h, out_w;
  int32_t kernel, stride, pad;
  const float *weight;
  const float *bias;
} cv_layer;

typedef struct cv_bound cv_bound;

/* Root intermediate bounds by per-layer CROWN (the bound of this library with
 * beta = 0, no splits, default alpha and specification [I; -I] on each ReLU
 * layer in turn), computed once per property as in App. B.1.
 *   layers[n_layers], ReLU after all but the last layer;
 *   x_lo, x_hi: host [n_props][d0] box;
 *   l_out, u_out: host [n_props][sum_{i<L} d_i], layer-major.
 * Synchronous.  Float32 arithmetic: the result is not outward-rounded. */
int cv_bound_root_bounds(const cv_layer *layers, int32_t n_layers, int32_t n_props,
                         const float *x_lo, const float *x_hi,
                         float *l_out, float *u_out, void *stream);

/* The same bounds made sound: each is evaluated as in sound mode (float64
 * with a rigorous rounding margin, rounded outward to float; each layer's
 * bounds built on the previous layers' sound bounds), so l_out and u_out
 * enclose every pre-activation the network takes on the box.  Same
 * arguments and behaviour as cv_bound_root_bounds. */
int cv_bound_root_bounds_sound(const cv_layer *layers, int32_t n_layers, int32_t n_props,
                               const float *x_lo, const float *x_hi,
                               float *l_out, float *u_out, void *stream);

/* Optimised intermediate bounds (Sec. 3.3): as cv_bound_root_bounds, but
 * each of the 2 d_i bounds of layer i is maximised over its own alpha' (one
 * per unstable neuron of the layers below: the unshared form of Sec. 3.3;
 * no splits at the root, so no beta') by `iters` projected-Adam steps from
 * CROWN's default (learning rate lr_alpha, decay lr_decay per step), keeping
 * the best iterate; each layer is built on the optimised bounds of the layers
 * below.  Each bound is therefore at least as tight as CROWN's.  sound = 1
 * reports every bound as sound mode does (cv_bound_set_sound: float64 with a
 * rigorous rounding margin, rounded outward to float).
 * iters = 0 is cv_bound_root_bounds (sound = 0) or _sound (sound = 1).
 * CV_EINVAL on iters < 0, sound outside 0/1 or non-finite rates. */
int cv_bound_root_bounds_opt(const cv_layer *layers, int32_t n_layers, int32_t n_props,
                             const float *x_lo, const float *x_hi, int32_t iters,
                             float lr_alpha, float lr_decay, int32_t sound,
                             float *l_out, float *u_out, void *stream);

/* Build a handle for one batch of subdomains (Theorem 3.1 inputs).
 *   layers[n_layers]: the network; the last layer must be dense.
 *   x_lo, x_hi: host [n_props][d0] input box of each property (the L-inf ball
 *     of Sec. 2.1, possibly clipped).
 *   m, C: host [n_props][m][d_L] specification rows, merged into the last
 *     layer (Sec. 2.1).
 *   l, u: host [n_props][sum_{i<L} d_i] intermediate bounds, layer-major;
 *     both NULL: computed here by per-layer CROWN on the GPU, exactly as
 *     cv_bound_root_bounds (float32, not outward-rounded; for sound mode
 *     pass cv_bound_root_bounds_sound's bounds instead).
 *   n_dom, dom_prop: host [n_dom] property of each subdomain.
 *   split_ptr: host [n_dom+1] CSR offsets; split_layer (1..L-1),
 *     split_neuron, split_side (+1: z >= 0, i.e. Z+, S = -1; -1: z < 0,
 *     i.e. Z-, S = +1), each host [nnz] (Eq. S).
 * CV_ESPLIT when a split names a layer or neuron out of range, a neuron that
 * is not root-unstable for its property, the same neuron twice in one
 * subdomain, a side other than +-1, or when nnz reaches 2^29.  CV_ESHAPE when
 * shapes do not chain, the last layer is a convolution, or a convolution has
 * a stride above 8, more than 128 columns in one of its implicit GEMMs
 * (stride^2 * in_c for the back-substitution, out_c forward), or rows,
 * tables and weights too large for a workgroup's 64 KB of LDS.
 * CV_EINVAL for non-finite inputs, x_lo > x_hi or a property index out of
 * range.  Validation happens before any device call.  n_dom = 0 is an empty
 * batch: every later call on the handle returns CV_OK without device work,
 * and its bound outputs may be NULL.
 * Synchronous; copies everything it needs to the device. */
int cv_bound_init(cv_bound **out, const cv_layer *layers, int32_t n_layers,
                  int32_t n_props, const float *x_lo, const float *x_hi,
                  int32_t m, const float *C, const float *l, const float *u,
                  int32_t n_dom, const int32_t *dom_prop, const int64_t *split_ptr,
                  const int32_t *split_layer, const int32_t *split_neuron,
                  const int8_t *split_side, void *stream);

/* Sizes of the caller-owned arrays: alpha entries, beta entries (nnz*m),
 * bound rows (n_dom*m).  Any output pointer may be NULL. */
int cv_bound_sizes(const cv_bound *h, int64_t *n_alpha, int64_t *n_beta, int64_t *n_rows);

/* Index of alpha for (subdomain, spec row, ReLU layer 1..L-1, neuron) in the
 * alpha layout, or -1 when that neuron is not root-unstable. Host only. */
int64_t cv_bound_alpha_offset(const cv_bound *h, int32_t dom, int32_t row, int32_t layer,
                              int32_t neuron);

/* CROWN's default lower slope (alpha = 1 where u >= -l, else 0) into every
 * alpha entry.  alpha: device [n_alpha]. */
int cv_bound_alpha_init(cv_bound *h, float *alpha, void *stream);

/* Bound g(alpha, beta) of Eq. beta_crown_lp (box form) for every row.
 * alpha: device [n_alpha] in [0,1]; beta: device [nnz*m] >= 0 (values are
 * used as given); lb: device [n_rows] output. */
int cv_bound_eval(cv_bound *h, const float *alpha, const float *beta, float *lb, void *stream);

/* Bound and its supergradient with respect to alpha and beta (reverse sweep
 * from the box minimiser x*; per-row, so d(sum lb)/d(var) = d(own row)/d(var)).
 * lb [n_rows], g_alpha [n_alpha], g_beta [nnz*m]: device outputs. */
int cv_bound_grad(cv_bound *h, const float *alpha, const float *beta, float *lb,
                  float *g_alpha, float *g_beta, void *stream);

/* cv_bound_grad for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation.
 * Same arguments, results and stream semantics as cv_bound_grad, but no call
 * allocates: where cv_bound_grad uses (and on its first call allocates) the
 * handle's workspace -- the two activation buffers, the per-row partial
 * sums, the stored A at unstable neurons, the box minimiser x* and the
 * sound-mode / l2-ball partials -- this call carves them from one static
 * device array of 32 MiB per GPU (its address resolved at cv_bound_init;
 * the array lives until the process ends).  CV_ENOMEM, with the bytes
 * needed in cv_last_error(), when the batch needs more than the array holds
 * (about R (2 w + 2 d0/8 + 1 + slots) + 4 n_alpha bytes for R = n_dom * m
 * rows of width w, plus 4 R d0 for a dense first layer).  Every piece is
 * written before it is read, so nothing carries over between calls, but all
 * calls on one GPU share the array: calls that overlap in time on the same
 * GPU (two streams, two threads, two handles) race and must be serialised
 * by the caller. */
int cv_bound_grad_noalloc(cv_bound *h, const float *alpha, const float *beta, float *lb,
                          float *g_alpha, float *g_beta, void *stream);

/* The primal side of the branch-and-bound step (Alg. 1 and its footnote; the
 * appendix on infeasible subdomains): for each row, the box minimiser x* of
 * the final linear function of the bound at (alpha, beta) (Eq.
 * beta_crown_linear over the box: x_lo where A(0) > 0, x_hi where A(0) < 0,
 * the centre where A(0) = 0), and the network itself evaluated at x*:
 *   ub[r]  = (C_p f(x*))_k, f with its exact ReLUs.  x* lies in the box, so
 *            ub bounds min over the box of (C_p f(x))_k from above; ub < 0 is
 *            a counter-example to that specification row;
 *   sat[r] = 1 if x* meets every split of the row's subdomain (z >= 0 for a
 *            z >= 0 split, z <= 0 for a z < 0 split), else 0.  Where 1, ub
 *            also bounds the subdomain's own minimum from above, so lb <= ub
 *            up to float32 rounding;
 *   lb[r]  = the bound itself (as cv_bound_eval), or skipped when lb is null.
 * alpha, beta as for cv_bound_eval; lb, ub [B*m] float32, sat [B*m] int32,
 * device buffers owned by the caller, written in stream order on `stream`.
 * Uses the per-layer kernels (and the back-substitution plan of
 * cv_bound_set_plan).  CV_EINVAL on a null ub, sat or required variable. */
int cv_bound_upper(cv_bound *h, const float *alpha, const float *beta, float *lb, float *ub, int32_t *sat,
                   void *stream);

/* Projected Adam ascent (Kingma & Ba; beta1 0.9, beta2 0.999, eps 1e-8) on
 * alpha in [0,1] and beta >= 0 for `iters` steps; step t (0-based, counted
 * from step0) uses learning rate lr * lr_decay^t and bias corrections of step
 * t+1.  Iterate k is evaluated before its step; the final iterate once more.
 *   alpha, beta: device in/out (start point in, final iterate out);
 *   adam_state: device [2*n_alpha + 2*n_beta] (first moments of alpha, second
 *     of alpha, first of beta, second of beta), in/out, or NULL for zero
 *     moments kept internally; step0: steps already taken (0 for a fresh run);
 *   lb_best: device [n_rows] out, max over the iters+1 evaluated bounds;
 *   lb_last: device [n_rows] out (may be NULL), bound of the final iterate.
 * The first call with a given set of arguments issues the loop's launches
 * directly; the second captures the whole loop in a HIP graph, which later
 * calls with the same arguments replay (a handle optimised once, as in a
 * branch-and-bound round, pays no capture). */
int cv_bound_optimize(cv_bound *h, int32_t iters, float lr_alpha, float lr_beta, float lr_decay,
                      float *alpha, float *beta, float *adam_state, int32_t step0,
                      float *lb_best, float *lb_last, void *stream);

/* Time the candidate tile shapes of every layer's kernels on this handle's
 * shapes and keep the fastest (process-wide cache keyed by shape): the GEMM
 * tilings of the dense layers, the kernel variants of the conv layers
 * (cv_bound_set_conv_variant), per layer and direction, and the fused dense
 * chain against per-layer kernels.  Synchronous.  Results do not depend on
 * the choice beyond float32 rounding of the summation order. */
int cv_bound_autotune(cv_bound *h, void *stream);

/* Execution plan of the dense layers at the top of the network, for the
 * back-substitution (chain_bwd) and the adjoint (chain_fwd): 1 runs the run of
 * dense layers as one fused kernel (each workgroup keeps its rows on chip
 * through all of them), 0 one kernel per layer.  cv_bound_init starts with
 * per-layer kernels, cv_bound_autotune makes a measured choice; this call
 * overrides both.  CV_EINVAL for other values, or for 1
 * where the network has no chain (its dense tail is missing, wider than 256
 * neurons, or does not fit the on-chip memory).  Results agree across plans
 * up to float32 summation order. */
int cv_bound_set_plan(cv_bound *h, int32_t chain_bwd, int32_t chain_fwd);

/* A new batch of subdomains for the handle (Alg. 1: each round bounds the
 * children of the subdomains it split), over the same network, properties,
 * specifications, root bounds, input sets and modes (sound mode, l_p balls,
 * forced tilings and conv variants, the sub-batch count set by
 * cv_bound_set_parts).  Arguments as cv_bound_init's n_dom .. split_side
 * (host pointers, copied; the same validation: CV_ESPLIT / CV_EINVAL leave
 * the handle's previous batch in place).  Batch-sized device buffers are
 * reused when the new batch is no larger than one the handle has held, else
 * reallocated with a quarter to spare (CV_ENOMEM then leaves the handle
 * without a batch: update it again or destroy it).  The alpha and beta
 * layouts follow the new batch (query cv_bound_sizes); the optimiser's graph
 * and any joint-optimisation state are dropped (a later
 * cv_bound_optimize_joint rebuilds it).  Synchronous on `stream` (it waits
 * for the device before it frees buffers). */
int cv_bound_update(cv_bound *h, int32_t n_dom, const int32_t *dom_prop, const int64_t *split_ptr,
                    const int32_t *split_layer, const int32_t *split_neuron, const int8_t *split_side,
                    void *stream);

/* Joint optimisation of intermediate-layer bounds (Sec. 3.3, Eq.
 * opt_non_convex).  As cv_bound_optimize, except that every subdomain's
 * pre-activation bounds of ReLU layers 2..L-1 are recomputed in each
 * iteration: layer i's are Theorem 3.1's bounds of z(i) (and of -z(i)) on the
 * sub-network of layers 1..i under the subdomain's splits below layer i, with
 * variables alpha', beta' of their own, shared by all neurons of layer i per
 * bound side (per subdomain: one alpha' entry per root-unstable neuron below
 * layer i, one beta' per split below it).  The tighter of the computed and
 * the root bound feeds the relaxation of the layers above (the gradient
 * follows the computed one unless it is looser than the root's by more than
 * 1e-4 max(1, |root|), so a tie carries it);
 * layer 1's bounds stay the root's (exact over the box).  All variables
 * ascend sum g together by projected Adam -- the gradient reaches alpha',
 * beta' through the bounds -- with lr_alpha for alpha and alpha', lr_beta for
 * beta and beta', lr * lr_decay^t at iteration t; alpha' starts at CROWN's
 * slope of the root bounds, beta' at 0, every Adam moment at 0.  A split
 * decides its neuron's relaxation whatever the bounds say (they contradict it
 * only for an empty subdomain).
 *   alpha, beta: device, in: the final objective's start (layouts as for
 *     cv_bound_optimize), out: its final iterate;
 *   lb_best: device [B][m], the best bound of the iters + 1 evaluated iterates;
 *   lb_last: device [B][m] or NULL, the final iterate's bound;
 *   l_out, u_out: device [B][sum d_i] or NULL, each subdomain's bounds of the
 *     final iterate (layer-major).
 * Boxes and plain float32 only: CV_EINVAL with sound mode on or l_p balls set.
 * The first call builds, per intermediate layer i, a pass of 2 d_i rows per
 * subdomain with per-row copies of its variables (device memory grows with
 * B x sum_i 2 d_i x the unstable neurons below layer i; CV_ENOMEM when it
 * does not fit), kept until cv_bound_destroy.  Eager on `stream` (no graph);
 * cv_bound_set_parts does not apply. */
int cv_bound_optimize_joint(cv_bound *h, int32_t iters, float lr_alpha, float lr_beta, float lr_decay,
                            float *alpha, float *beta, float *lb_best, float *lb_last, float *l_out,
                            float *u_out, void *stream);

/* The shared variables of intermediate layer `layer` (2..L-1) after the last
 * cv_bound_optimize_joint: alpha' and beta' of its final iterate and their
 * gradients of that call's last iteration (zeros when it ran no iteration).
 * Layouts, per subdomain in order: alpha' [2][uc_b] -- lower-bound side, then
 * upper-bound side; uc_b = root-unstable neurons of b's property in layers
 * 1..layer-1, in layer-major index order (the order of the handle's alpha
 * blocks) -- and beta' [nnz_layer][2]: the subdomain's splits on layers below
 * `layer`, in their CSR order, each with (lower side, upper side).
 * cv_bound_joint_sizes gives the two lengths.  Outputs are device buffers;
 * any may be NULL; stream-ordered copies.  CV_EINVAL before the first
 * cv_bound_optimize_joint or for a layer outside 2..L-1. */
int cv_bound_joint_sizes(const cv_bound *h, int32_t layer, int64_t *n_alpha_p, int64_t *n_beta_p);
int cv_bound_joint_vars(cv_bound *h, int32_t layer, float *alpha_p, float *beta_p, float *g_alpha_p,
                        float *g_beta_p, void *stream);

/* Concurrent sub-batches of cv_bound_optimize: the subdomains are split into
 * nparts contiguous ranges of nearly equal size, each optimised by its own
 * captured graph on its own stream, forked from and joined back into the
 * caller's stream (the kernels of one range fill the gaps and tails of the
 * other's).  Results are those of the same algorithm per subdomain; the
 * float32 summation order may differ from one range to another.  1 disables
 * the split.  cv_bound_init chooses 2 for batches of 4096 rows or more, else
 * 1.  CV_EINVAL outside 1..4; more parts than subdomains are reduced. */
int cv_bound_set_parts(cv_bound *h, int32_t nparts);

/* GEMM tilings of the dense-layer kernels (back-substitution, Theorem 3.1's
 * A(i-1) = Lambda(i) W(i), and the adjoint's forward steps): tile shape, K
 * slab and how many slabs of global loads are kept in flight.  Every tiling
 * computes the same result up to float32 summation order.
 * cv_bound_num_tilings: how many there are (numbered from 0).
 * cv_bound_set_tiling: force tiling `tiling` on every dense layer of h (and
 * of its concurrent sub-batches) in both directions, or -1 to return to the
 * tuned choice per layer shape (cv_bound_autotune's, else a built-in
 * default).  A tiling that keeps all of K in flight cannot take a layer
 * deeper than it holds; such a layer runs a two-deep tiling instead.  A later
 * cv_bound_autotune replaces the forced choice.  CV_EINVAL outside
 * -1..cv_bound_num_tilings()-1. */
int32_t cv_bound_num_tilings(void);
int cv_bound_set_tiling(cv_bound *h, int32_t tiling);

/* Kernel variants of the conv layers (back-substitution through a conv
 * layer as a transposed convolution, Theorem 3.1's A(i-1) = Lambda(i) W(i),
 * and the adjoint's forward convolution), all computing the same result up
 * to float32 summation order:
 *   0  row-major: each workgroup takes one batch row at a time, the weight
 *      matrix held in LDS;
 *   1  row-major, the weights read from global memory (L1/L2);
 *   2  subdomain-major: each workgroup takes the specification rows of one
 *      subdomain in turn and keeps the subdomain's status records and its
 *      property's chords (or box) in registers across them, weights in LDS;
 *   3  subdomain-major, weights from global memory.
 * cv_bound_num_conv_variants: how many there are.
 * cv_bound_set_conv_variant: force `variant` on every conv layer of h (and of
 * its sub-batches) in both directions where it can run that layer (where it
 * cannot, the layer keeps its default), or -1 to return to the tuned choice
 * per layer shape (cv_bound_autotune's, else the default: subdomain-major
 * where an instantiation holds the layer's rows, weights in LDS up to 16 KB).
 * CV_EINVAL outside -1..cv_bound_num_conv_variants()-1.
 * cv_bound_conv_variant: the variant conv layer `layer` (1..L) runs in
 * direction dir (0 back-substitution, 1 adjoint), or -1 for a dense layer or
 * bad arguments.  Host only. */
int32_t cv_bound_num_conv_variants(void);
int cv_bound_set_conv_variant(cv_bound *h, int32_t variant);
int cv_bound_conv_variant(const cv_bound *h, int32_t layer, int32_t dir);

/* Sound mode (off by default): every bound this handle reports (eval, grad,
 * upper, optimize) is rigorous: it lies below the value the same relaxation
 * (same alpha, beta and sign decisions) gives in exact arithmetic, hence
 * below the true minimum (Theorem 3.1's bound is sound for any alpha in
 * [0,1], beta >= 0).  The bound is evaluated in float64 -- the specification
 * merged into the last layer, every back-substitution product, the
 * relaxation (chords formed in double from the root bounds), the constants
 * and the concretisation -- and lowered by a rigorous bound on its float64
 * rounding (per-row sum of |Lambda_k| times per-neuron weights computed once
 * on the host: g(d_i) sum |W| max|input|, the rounding of Lambda and of the
 * chord, every addition into the constant and the concretisation, the
 * merged specification; g(n) = n u/(1 - n u), u = 2^-52), then rounded down
 * to float: typically within one float ulp of the exact bound.
 * cv_bound_optimize runs its iterations with the plain float32 kernels,
 * records each row's best iterate (its float32 bound and its variables),
 * and reports lb_best = the larger of the float64 sound bounds of that
 * iterate and of the final one, lb_last = the final iterate's.  Gradients
 * are those of the bound itself.  on: 0 or 1 (else CV_EINVAL).  Switching
 * on computes the weights for the current input sets, boxes or the balls of
 * cv_bound_set_input_l2 (host work, synchronous on `stream`) and allocates
 * the float64 buffers; CV_ESHAPE if a ReLU layer is wider than 8192. */
int cv_bound_set_sound(cv_bound *h, int32_t on, void *stream);

/* l2-ball input sets (Sec. 2.1 allows any l_p ball; Theorem 3.1's last step
 * then concretises with the dual norm): property p's input set becomes
 * {x : ||x - x0_p||_2 <= eps_p} in place of its box.  The bound's last step
 * is then A(0) x0 - eps ||A(0)||_2 (row of A(0) = Lambda(1) W(1)), and the
 * adjoint and cv_bound_upper use its minimiser x* = x0 - eps A(0)/||A(0)||_2
 * (x0 where A(0) = 0).  The handle's root bounds must hold over the balls
 * (the caller's responsibility, as for boxes).
 *   x0: host [n_props][d0], finite; eps: host [n_props], finite and >= 0;
 *   x0 = NULL returns every property to its box (eps ignored).
 * Applies to the handle and its sub-batches, now and when later created.
 * With sound mode on, the margin is rebuilt for the balls (an input
 * coordinate is bounded by |x0_j| + eps_p), and the bound is lowered by an
 * upper bound on eps ||A(0)||_2 and by the rounding of the A(0) x0 sum
 * (g ||A(0)||_2 ||x0||_2).  The fused dense chain is not used over balls.
 * Copies its arguments (synchronous on `stream`); the first call allocates
 * per-row buffers (CV_ENOMEM).  W(1) x0 + b(1) is formed on the host in
 * double and rounded once. */
int cv_bound_set_input_l2(cv_bound *h, const float *x0, const float *eps, void *stream);

/* l_p-ball input sets for any p in [4/3, inf) (Sec. 2.1's l_p balls; Eq.
 * beta_crown_lp concretises with the dual norm, 1/p + 1/q = 1): property
 * k's input set becomes {x : ||x - x0_k||_p <= eps_k}.  The bound's last
 * step is A(0) x0 - eps ||A(0)||_q, and the adjoint and cv_bound_upper use
 * the minimiser x* = x0 - eps sign(A(0)) |A(0)|^(q-1) / ||A(0)||_q^(q-1)
 * (x0 where A(0) = 0), the equality case of Hoelder's inequality.
 * p = 2 is exactly cv_bound_set_input_l2; the box (p = inf) is the handle's
 * x_lo, x_hi (x0 = NULL returns to it).  q <= 4 (p >= 4/3) keeps the float32
 * powers |A(0)|^q in range for entries of magnitude about 1e-9 .. 1e9; the
 * powers are formed as 2^(q log2|a|).  Arguments, allocation, sub-batches
 * and the caller's duty for root bounds as for cv_bound_set_input_l2.
 * CV_EINVAL for p < 4/3 or not finite, and for p != 2 while sound mode is
 * on (cv_bound_set_sound likewise refuses to switch on over such balls). */
int cv_bound_set_input_lp(cv_bound *h, const float *x0, const float *eps, float p, void *stream);

/* Per-kernel timing of one gradient pass plus one plain evaluation, issued
 * eagerly on `stream`, repeated `reps` times.  Each kernel launch of a pass
 * is issued 8 times back to back (same arguments) between two HIP events on
 * `stream`; a launch is timed as elapsed / 8.  Fills up to
 * max_out records; *n_out gets the number of distinct kernels.  flops and
 * bytes are algorithmic counts: the multiply-adds (x2) of the contraction a
 * launch performs, and the bytes it must read and write at least once. */
typedef struct cv_kernel_stat {
  char name[64];
  int32_t launches;     /* launches per pass                              */
  double total_ms;      /* per-launch time, summed over launches and reps */
  double flops;         /* algorithmic flops, summed over launches per rep */
  double bytes;         /* algorithmic HBM bytes, summed likewise          */
} cv_kernel_stat;
int cv_bound_profile(cv_bound *h, const float *alpha, const float *beta, int32_t reps,
                     cv_kernel_stat *out, int32_t max_out, int32_t *n_out, void *stream);

void cv_bound_destroy(cv_bound *h);
const char *cv_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* CVBOUND_H */
