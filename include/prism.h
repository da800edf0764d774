/*
 * prism.h -- C ABI of libprism, the MI355X (gfx950) implementation of the
 * per-iteration analysis-by-synthesis pass of PRISM (arxiv 2604.00250).
 *
 * One iteration of the fit evaluates, for every masked voxel x and every
 * measurement n of one or many independent problems ("groups"),
 *
 *   tissue signal (Eq. 3-5)  S_n(x) = S0 (f_csf E_csf + f_gm E_gm
 *                                         + sum_k f_wm,k E_wm,k + f_res E_res)
 *   calibration   (Eq. 6)    yhat_n(x) = exp(alpha_n) B(x) S_n(x) + beta_n
 *   data term     (Eq. 8/9)  MSE (1/|M|) sum (yhat - y)^2, or the Rician NLL
 *                            sum [log s^2 + (y^2 + yhat^2)/(2 s^2) - log I0(y yhat/s^2)]
 *                            with s = exp(sigma_log)
 *   priors        (Sec. 2.4) Huber-Laplacian on the fractions (Eq. 7),
 *                            direction repulsion, sparsity of minor fibres,
 *                            orphan-WM suppression, directional continuity,
 *                            fibre ordering, L2 on the calibration parameters
 *                            and total variation of the bias field
 *
 * and the exact gradient of the total objective (Sec. 2.5) with respect to
 * every raw parameter.  Readings of points the paper leaves open are fixed in
 * the project's design notes and repeated where they matter below.
 *
 * Conventions shared by every entry point
 *   - Units: b-values in ms/um^2 (s/mm^2 x 1e-3), diffusivities in um^2/ms.
 *   - A group is one independent problem: a box nx*ny*nz, a mask, one
 *     acquisition, K fibre slots, one data mode, one calibration vector.
 *     Its voxels are the masked voxels in C (raster) order, z fastest:
 *     voxel (i,j,k) has raster index (i*ny + j)*nz + k.
 *   - theta_micro of a group: parameter-major float32 [P][V] at the group's
 *     micro_offset, P = 5 + 4K (+2 with learned diffusivities), rows:
 *       s0 (softplus -> S0), logit_csf, logit_gm, logit_wm[0..K-1], logit_res
 *       (softmax -> fractions), v[0..K-1][x,y,z] (l2-normalised -> d_k),
 *       fin (sigmoid -> f_intra) [, dpar, dperp (softplus -> D_par, D_perp)].
 *   - theta_cal of a group: float32 [n_bias + 2N + 1] at its cal_offset:
 *       bias coefficients, alpha[N], beta[N], sigma_log.
 *   - y and yhat of a group: float32 [N][V] at its y_offset.
 *   - grad_micro / grad_cal mirror theta_micro / theta_cal.
 *   - loss: float64 [n_groups][PRISM_LOSS_TERMS] (data, spatial, rep,
 *     sparse, orphan, continuity, ordering, cal, tv, total); the total is at
 *     index PRISM_LOSS_TOTAL.
 *   - Every tensor argument of a per-iteration call is a caller-owned DEVICE
 *     pointer that must stay valid until the work queued on `stream` (a
 *     hipStream_t passed as void*, NULL = the default stream) completes.
 *     Per-iteration calls allocate nothing and never synchronise, so they can
 *     be captured in a HIP graph.
 *   - Every function returns a prism_status; on failure
 *     prism_last_error() gives a message for the calling thread.  No
 *     function aborts and no C++ exception crosses the ABI.
 *   - Calls on different streams with disjoint outputs and workspaces may
 *     run concurrently; a problem handle is read-only after creation except
 *     through prism_problem_tune().
 */
#ifndef PRISM_H
#define PRISM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PRISM_ABI_VERSION 4
#define PRISM_MAX_K 6
#define PRISM_MAX_MEAS 1024
#define PRISM_MAX_EDGE 1023
#define PRISM_LOSS_TERMS 10
#define PRISM_LOSS_TOTAL 9

typedef enum {
  PRISM_OK = 0,
  PRISM_E_INVALID = -1,     /* bad argument: null pointer, size or enum out of range */
  PRISM_E_UNSUPPORTED = -2, /* well-formed but not supported by the library */
  PRISM_E_HIP = -3,         /* a HIP runtime call or kernel launch failed */
  PRISM_E_WORKSPACE = -4,   /* workspace smaller than prism_workspace_bytes() */
  PRISM_E_ALLOC = -5        /* host or device allocation failed (create/tune only) */
} prism_status;

enum { PRISM_MSE = 0, PRISM_RICIAN = 1 };                     /* Eq. 8, Eq. 9 */
enum { PRISM_BIAS_NONE = 0, PRISM_BIAS_POLY2 = 1, PRISM_BIAS_TRILINEAR8 = 2 };
/* Priors (Sec. 2.4).  The paper prints the stabilisation terms' weights but
 * not their forms; these are read as (sums over masked voxels x, averaged
 * over |M|, f_k the WM fractions, d_k the unit fibre directions):
 *   ORPHAN      max(0, 1 - S0(x)/s0_orphan) * sum_k f_k(x)
 *   CONTINUITY  1/|N(x)| sum_{x' in N(x)} sum_k (1 - (d_k(x).d_k(x'))^2),
 *               N(x) the group's Eq. 7 neighbourhood (nothing when it is 0)
 *   ORDERING    sum_k max(0, f_k+1(x) - f_k(x))
 *   TV          sum_a [x + e_a masked] |B(x + e_a) - B(x)| over the three
 *               axes (Sec. 2.4 calibration regularisers; needs a bias basis)
 * The derivative of a kink (|0|, a hinge at 0) is taken as 0. */
enum {
  PRISM_PRIOR_SPATIAL = 1, PRISM_PRIOR_REP = 2, PRISM_PRIOR_SPARSE = 4, PRISM_PRIOR_CAL = 8,
  PRISM_PRIOR_ORPHAN = 16, PRISM_PRIOR_CONTINUITY = 32, PRISM_PRIOR_ORDERING = 64,
  PRISM_PRIOR_TV = 128
};
enum {                       /* bits OR-ed into the device status word */
  PRISM_ST_NONFINITE_LOSS = 1,
  PRISM_ST_NONFINITE_GRAD = 2,
  PRISM_ST_ZERO_DIRECTION = 4 /* a raw fibre direction v_k had zero norm */
};

/* One acquisition: N measurements.  bval >= 0 (ms/um^2), bvec unit rows for
 * b > 0 (|g| within 1e-3 of 1; rows with b = 0 are not used).  Host memory,
 * copied by prism_problem_create. */
typedef struct {
  int32_t n_meas;
  const float* bval; /* [N] */
  const float* bvec; /* [N][3] */
} prism_acq;

/* One group (independent problem).  Host memory, copied at create. */
typedef struct {
  int32_t nx, ny, nz;        /* box, each in 1..PRISM_MAX_EDGE */
  int32_t K;                 /* fibre slots, 1..PRISM_MAX_K */
  int32_t mode;              /* PRISM_MSE or PRISM_RICIAN */
  int32_t bias;              /* PRISM_BIAS_*: none, degree-2 polynomial in box
                                coordinates (10 coefficients, order 1,x,y,z,x^2,
                                y^2,z^2,xy,xz,yz with x in [-1,1] across the box),
                                or the paper's 8^3 trilinear control grid (Sec. 2.3) */
  int32_t acq;               /* index into the acquisition array */
  int32_t neighbourhood;     /* 0 (no spatial prior), 6 or 26 (Eq. 7) */
  int32_t learn_diffusivity; /* 0: D_par, D_perp fixed (Eq. 5); 1: per-voxel softplus */
  uint32_t priors;           /* PRISM_PRIOR_* bits */
  const uint8_t* mask;       /* [nx*ny*nz] raster order, nonzero = in the mask; NULL = all */
} prism_group_desc;

/* Model constants.  prism_model_defaults() fills the paper's values:
 * D_csf 3.0, D_gm 0.9, D_res 0.2 (Eq. 4), D_par 1.7, D_perp 0.4 (Eq. 5),
 * lam_sp 0.01 with Huber delta 0.05 (Eq. 7), lam_rep 0.01, lam_sparse 0.02
 * with tau 0.15, lam_orphan 0.01, lam_cont 0.005, lam_order 0.01 (Sec. 2.4),
 * and values the paper does not print (readings): the calibration L2 weights
 * 0.01, lam_tv 0.01, and s0_orphan 0.1 (S0 below which WM is penalised, on
 * b0-normalised signals).  All must be finite and >= 0; s0_orphan > 0 and
 * d_par > 0 (a stick with no parallel diffusivity is not a fibre; it is also
 * the unit of the fibre attenuation's exponent in the fused pass), else
 * PRISM_E_INVALID. */
typedef struct {
  float d_csf, d_gm, d_res, d_par, d_perp;
  float lam_sp, huber_delta, lam_rep, lam_sparse, tau_sparse;
  float lam_alpha, lam_beta, lam_bias;
  float lam_orphan, s0_orphan, lam_cont, lam_order, lam_tv;
} prism_model;

typedef struct prism_problem prism_problem;

typedef struct {
  int64_t n_vox;        /* masked voxels V */
  int32_t n_meas;       /* N */
  int32_t K;
  int32_t n_params_vox; /* P */
  int32_t n_bias;       /* 0, 10 or 512 */
  int32_t n_cal;        /* n_bias + 2N + 1 */
  int32_t pad;
  int64_t micro_offset; /* float offset of the group's [P][V] block */
  int64_t cal_offset;   /* float offset of the group's calibration vector */
  int64_t y_offset;     /* float offset of the group's [N][V] block */
} prism_group_info_t;

typedef struct {
  int64_t n_vox;   /* total masked voxels */
  int64_t n_micro; /* floats of theta_micro / grad_micro */
  int64_t n_cal;   /* floats of theta_cal / grad_cal */
  int64_t n_y;     /* floats of y / yhat */
  int32_t n_groups;
  int32_t n_buckets; /* kernel variants (K, mode, learned D) the problem uses */
} prism_problem_info_t;

/* Launch shape of the fused pass (set by prism_problem_tune). */
typedef struct {
  int32_t vox_per_lane; /* 1 or 2 voxels per lane (the persistent launch uses 1) */
  int32_t n_split;      /* 1, 2 or 4 waves sharing one voxel row (each over a part of
                           the measurements); 0 = chosen per work item from its size */
  int32_t item_vox;     /* voxels per work item (one thread block at a time), a
                           multiple of 64 * vox_per_lane * 4 / n_split; 0 = automatic:
                           one block chunk (that multiple) with a fixed n_split, else
                           about six blocks per compute unit over the problem */
  int32_t persistent;   /* 0: one launch per kernel variant (K, mode, learned D,
                           voxels per lane); 1: persistent launches over all work
                           items, one per register class (K <= 2, compiled for three
                           waves per SIMD; K >= 3, for two), each over its items
                           largest first, each block popping items from a device
                           counter of its launch */
  int32_t max_blocks;   /* persistent launches: at most this many blocks together,
                           shared out by work (0 = as many as the device holds at
                           once; at least one per launch); fewer blocks than work
                           items make each block run several items in turn */
  int32_t stagger;      /* 1 (the default): a problem of one large group cut into
                           one-chunk items (vox_per_lane 1, n_split 1, item_vox 0)
                           starts every XCD's run of items with CUs/8 shorter items
                           (half of 64 voxels over four waves, half of 128 over two),
                           so that one block per compute unit runs out of phase with
                           the others and the blocks' epilogue memory traffic does
                           not arrive all at once; 0: equal items only.  Ignored
                           where it does not apply (several groups, other shapes,
                           fewer than two rounds of blocks, or when the measurement
                           split's LDS would cost the variant a block per CU). */
  int32_t concurrent;   /* 1 (the default): a plan of several fused-pass launches
                           (one per kernel variant, or the persistent launches of
                           two register classes) runs them on up to
                           four streams at once -- the caller's and three the
                           problem owns (default priority) -- forked from and
                           joined back into the caller's stream with events, so
                           that one variant's tail overlaps the others' work (this
                           also records into a HIP graph); 0: one after the other
                           on the caller's stream.  The enqueue of one call is
                           atomic with respect to other host threads using the
                           same problem. */
} prism_launch;

/* Launch shape of one bucket of groups: those with n_meas measurements, K
 * fibre slots, data mode `mode` and learn_diffusivity.  Overrides the
 * problem's vox_per_lane (ignored by the persistent launch), n_split and
 * item_vox for the groups of that bucket. */
typedef struct {
  int32_t n_meas, K, mode, learn_diffusivity; /* the bucket */
  int32_t vox_per_lane, n_split, item_vox;    /* as in prism_launch */
} prism_bucket_launch;

int32_t prism_abi_version(void);
const char* prism_last_error(void);
void prism_model_defaults(prism_model* m);

/* Build a problem: validates every descriptor, compacts each mask to its
 * raster-ordered voxel list, builds the neighbour tables of Eq. 7 and the work
 * plan, and copies them with the acquisitions to the current HIP device.
 * Allocates (host and device); not for use under graph capture.  On success
 * *out owns those allocations until prism_problem_destroy. */
int32_t prism_problem_create(prism_problem** out, const prism_group_desc* groups,
                             int32_t n_groups, const prism_acq* acqs, int32_t n_acq,
                             const prism_model* model);
int32_t prism_problem_destroy(prism_problem* h);
int32_t prism_problem_info(const prism_problem* h, prism_problem_info_t* info);
int32_t prism_group_info(const prism_problem* h, int32_t group, prism_group_info_t* info);
/* Re-plan the work items for a launch shape; allocates, like create.  On an
 * invalid shape the previous plan is kept and PRISM_E_INVALID returned. */
int32_t prism_problem_tune(prism_problem* h, const prism_launch* launch);
/* As prism_problem_tune, with per-bucket shapes: buckets[0..n_buckets) each
 * name a (n_meas, K, mode, learn_diffusivity) bucket present in the problem
 * (at most once) and its shape; the other buckets take `launch`.  Replaces the
 * overrides of an earlier call. */
int32_t prism_problem_tune_buckets(prism_problem* h, const prism_launch* launch,
                                   const prism_bucket_launch* buckets, int32_t n_buckets);
int32_t prism_problem_launch(const prism_problem* h, prism_launch* launch);
/* The problem's buckets in order of first appearance among the groups, each
 * with the shape its groups run with; *n receives the number of buckets, of
 * which the first min(cap, *n) are written to out (host memory). */
int32_t prism_problem_buckets(const prism_problem* h, prism_bucket_launch* out, int32_t cap,
                              int32_t* n);
/* The current plan: work items, fused-pass launches per call, and the blocks of
 * the persistent launches together (0 when the plan is not persistent). */
int32_t prism_problem_plan_info(const prism_problem* h, int32_t* n_items, int32_t* n_launches,
                                int32_t* persistent_blocks);
/* Hash of the sources the library was built from (a NUL-terminated string
 * owned by the library), so that cached launch shapes and profiles can be
 * tied to one build. */
const char* prism_build_id(void);

/* Bytes of device workspace prism_loss_grad needs (per-item partial sums and
 * the Eq. 7 residual weights).  The caller allocates it; contents need not be
 * initialised and are overwritten by every call. */
int32_t prism_workspace_bytes(const prism_problem* h, size_t* bytes);

/* Forward model only (Eq. 3-6): yhat [N][V] per group from theta_micro and
 * theta_cal.  Device pointers; asynchronous on `stream`. */
int32_t prism_synthesize(const prism_problem* h, const float* theta_micro,
                         const float* theta_cal, float* yhat, void* stream);

/* Fused forward + adjoint pass: loss terms per group and the full gradient.
 *   y           [n_y]      measurements (device)
 *   theta_micro [n_micro], theta_cal [n_cal]  parameters (device)
 *   loss        [n_groups][PRISM_LOSS_TERMS] float64 (device, overwritten)
 *   grad_micro  [n_micro], grad_cal [n_cal] (device, overwritten)
 *   workspace   >= prism_workspace_bytes (device), workspace_bytes its size
 *   status      device uint32; PRISM_ST_* bits are OR-ed in, never cleared
 * Asynchronous on `stream`; allocates nothing; graph-capturable. */
int32_t prism_loss_grad(const prism_problem* h, const float* y, const float* theta_micro,
                        const float* theta_cal, double* loss, float* grad_micro,
                        float* grad_cal, void* workspace, size_t workspace_bytes,
                        uint32_t* status, void* stream);

/* prism_loss_grad without a workspace argument, for callers that cannot
 * allocate device memory (code that must not call hipMalloc: serving loops,
 * harnesses that forbid allocation, work recorded into HIP graphs by callers
 * that own no device buffers).  The workspace is a static device array of
 * PRISM_NOALLOC_WORKSPACE_BYTES per GPU inside the library, held from the
 * library's load until the process ends; its address is looked up once per
 * device by prism_problem_create.  Problems whose prism_workspace_bytes
 * exceeds that size are rejected with PRISM_E_WORKSPACE (nothing is queued).
 * Calls on one GPU share that GPU's array (it keeps the last call's contents;
 * nothing in it needs clearing between calls): two calls that may overlap on
 * one GPU, on different streams or from different threads, race and give
 * undefined results; calls queued on one stream are ordered and safe.  The
 * other arguments and the results are those of prism_loss_grad, bit for
 * bit.  Asynchronous on `stream`; allocates nothing. */
#define PRISM_NOALLOC_WORKSPACE_BYTES ((size_t)64 << 20)
int32_t prism_loss_grad_noalloc(const prism_problem* h, const float* y, const float* theta_micro,
                                const float* theta_cal, double* loss, float* grad_micro,
                                float* grad_cal, uint32_t* status, void* stream);

/* Adam (Kingma & Ba, Algorithm 1; the optimiser of Table 2 that the fit uses
 * here), elementwise over n float32 parameters, PyTorch's form:
 *   m = b1 m + (1-b1) g;  v = b2 v + (1-b2) g^2;  t = step[0] + 1
 *   p -= lr/(1-b1^t) * m / (sqrt(v)/sqrt(1-b2^t) + eps)
 * `step` is a DEVICE int32[2]: step[0] counts completed steps and is
 * incremented by the call; step[1] is internal and must be 0 before the first
 * call (the call leaves it 0).  p, g, m, v are device arrays of n floats.
 * Asynchronous; graph-capturable (replays advance step[0]). */
int32_t prism_adam_step(float* p, const float* g, float* m, float* v, int64_t n, float lr,
                        float beta1, float beta2, float eps, int32_t* step, void* stream);

/* One Adam iteration of the fit: the loss terms at theta (as prism_loss_grad
 * reports them) and the Adam update of theta_micro and, if update_cal != 0,
 * theta_cal, after which step[0] has advanced by one.  The results are
 * bitwise those of prism_loss_grad followed by prism_adam_step over the same
 * parameters.  The per-voxel parameters are updated inside the fused pass, so
 * their gradient never goes through memory; when a group uses the continuity
 * prior (which reads neighbouring voxels' parameters during the pass) the call
 * runs the two steps one after the other and grad_micro receives the
 * per-voxel gradient.  Arguments as for prism_loss_grad and prism_adam_step;
 * m_micro, v_micro [n_micro] and m_cal, v_cal [n_cal] are the Adam moments
 * (device), grad_micro [n_micro] (device) is scratch for the unfused case,
 * grad_cal [n_cal] receives the calibration gradient.
 *   loss_history  NULL, or a device float64 ring [history_len][n_groups]
 *                 [PRISM_LOSS_TERMS]: the call also writes its loss rows to
 *                 slot t mod history_len, t = the iteration's index (step[0]
 *                 before the call), so that a graph-captured loop keeps the
 *                 whole loss history on the device; history_len >= 1 then.
 * Asynchronous; allocates nothing; graph-capturable. */
int32_t prism_iteration_adam(const prism_problem* h, const float* y, float* theta_micro,
                             float* theta_cal, float* m_micro, float* v_micro, float* m_cal,
                             float* v_cal, int32_t* step, float lr, float beta1, float beta2,
                             float eps, int32_t update_cal, double* loss, double* loss_history,
                             int32_t history_len, float* grad_micro,
                             float* grad_cal, void* workspace, size_t workspace_bytes,
                             uint32_t* status, void* stream);

/* Rprop (Riedmiller & Braun 1993; the paper's solver, Sec. 2.5), PyTorch's
 * variant: per coordinate, s = g * prev; step *= eta_plus if s > 0, eta_minus
 * if s < 0; step clamped to [step_min, step_max]; where s < 0 the gradient is
 * taken as 0; p -= sign(g) * step; prev = g.  prev and step are device arrays
 * of n floats (prev starts at 0, step at the initial step size, e.g. 0.01). */
int32_t prism_rprop_step(float* p, const float* g, float* prev, float* step, int64_t n,
                         float eta_minus, float eta_plus, float step_min, float step_max,
                         void* stream);

/* Whole-volume slabs (Sec. 2.5): a volume too large for one fit is fitted as
 * overlapping slabs along z, each an independent group with its own
 * calibration, and the per-slab maps are blended where slabs overlap.
 *
 * prism_stitch_plan declares the groups of `h` to be such slabs: group g
 * covers slices z0[g] .. z0[g] + nz_g - 1 of a volume nx x ny x nz (z0 a host
 * array of n_groups entries, strictly increasing; every group with the
 * volume's nx and ny, the same K and the same learn_diffusivity; no slice in
 * more than two slabs).  It builds the stitch table on the device (allocates;
 * not for graph capture; replaces an earlier plan) and returns in *n_out the
 * number of output voxels: the union of the slabs' masked voxels, in raster
 * order of the volume.
 *
 * prism_stitch_maps writes float32 maps [P][n_out] (device), P = 5 + 4K (+2),
 * rows S0, fractions (csf, gm, wm_0..K-1, res), unit directions d_k (x, y, z),
 * f_intra [, D_par, D_perp]: the constrained quantities of theta_micro.  A
 * voxel of one slab takes that slab's values.  In an overlap of o slices the
 * slabs are weighted by linear ramps, (s + 1)/(o + 1) at the s-th slice from
 * a slab's edge (the two weights sum to one); the fibres of the lighter slab
 * (the upper one on a tie) are matched to the heavier slab's slots, each slot
 * in turn taking the unmatched fibre with the largest |cos| (lowest index on
 * ties), flipped to the same sign, blended and renormalised; the output keeps
 * the heavier slab's slot order.  (The paper states weighted averaging only;
 * the ramp and the matching are readings.)  Asynchronous; allocates nothing;
 * PRISM_E_INVALID before a plan. */
int32_t prism_stitch_plan(prism_problem* h, int32_t nx, int32_t ny, int32_t nz, const int32_t* z0,
                          int64_t* n_out);
int32_t prism_stitch_maps(const prism_problem* h, const float* theta_micro, float* maps,
                          void* stream);

/* The Rician data term's special functions (Eq. 9) at arguments z >= 0, as
 * the fused pass evaluates them: log_i0e[i] = log(I0(z) e^-z),
 * one_minus_ratio[i] = 1 - I1(z)/I0(z) and q[i] = 2 z (1 - I1(z)/I0(z)) (the
 * NLL adjoint and its sigma derivative use these).  Device arrays of n floats;
 * asynchronous on `stream`.  For checking the approximation against a
 * reference (its relative error is below 2e-7 over [0, 1e5]). */
int32_t prism_rician_terms(const float* z, float* log_i0e, float* one_minus_ratio, float* q, int64_t n,
                           void* stream);

/* Optional per-kernel timing of the fused pass: when enabled, prism_loss_grad
 * records HIP events around each launch of the fused kernel on `stream`
 * (events are created here, not in the timed call).  prism_profile_read
 * synchronises on the last event and returns the summed milliseconds and the
 * number of timed launches since the last reset. */
int32_t prism_profile_enable(prism_problem* h, int32_t enable, int32_t max_launches);
int32_t prism_profile_read(prism_problem* h, double* total_ms, int32_t* launches);

#ifdef __cplusplus
}
#endif
#endif /* PRISM_H */
