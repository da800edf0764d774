// Internal structures shared by the host planner (prism_host.cpp) and the
// kernels (prism_kernels.hip).  Not part of the C ABI.
#pragma once
#include <stdint.h>

#include <hip/hip_runtime.h>

namespace prism {

constexpr int kBlock = 256;          // threads per block of the fused pass (4 waves)
constexpr int kWave = 64;
constexpr int kMaxK = 6;
constexpr int kMaxC = kMaxK + 3;     // tissue compartments (csf, gm, wm_1..K, res)
constexpr int kAcqStride = 12;       // floats per staged measurement
constexpr int kRecHead = 19;         // record fields before alpha[N], beta[N]
// record field indices (float64)
enum RecField : int {
  kRecData = 0,     // data-term partial: MSE sum r^2, NLL sum of the positive parts
  kRecSpatial = 1,  // Huber-Laplacian partial (written by k_spatial)
  kRecRep = 2,      // repulsion partial
  kRecSparse = 3,   // sparsity partial
  kRecOrphan = 4,   // orphan-WM partial
  kRecCont = 5,     // directional-continuity partial
  kRecOrder = 6,    // fibre-ordering partial
  kRecTV = 7,       // bias-field total-variation partial
  kRecSigma = 8,    // NLL: sum of (r^2/s^2 + 2z(1-R)) (d/dsigma_log = 2N|M| - this)
  kRecBias = 9,     // 10 slots: sum_x phi_j(x) dlogB(x)
  kRecAlpha = kRecHead
};
constexpr int kLossTerms = 10;       // data, spatial, rep, sparse, orphan, continuity,
                                     // ordering, cal, tv, total

struct GroupDev {
  int64_t micro_off;  // float offset of theta_micro / grad_micro
  int64_t cal_off;    // float offset of theta_cal / grad_cal
  int64_t y_off;      // float offset of y / yhat
  int64_t vox_off;    // offset into per-voxel tables (coords)
  int64_t nbr_off;    // int32 offset of the neighbour table [ntab][V]; entries 0-5 are
                      // the face neighbours -x, +x, -y, +y, -z, +z, then the rest of 26
  int64_t ninv_off;   // float offset of 1/|N(x)| [V] (0 without neighbours)
  int64_t w_off;      // float offset of the spatial weights [V][C], then fractions [V][C], in the workspace
  int64_t glb_off;    // float offset of per-voxel dL/dlogB [V] in the workspace (trilinear)
  int64_t rec_off;    // float64 offset of the group's first item record
  int64_t grid_off;   // int32 offset of the dense raster->voxel index grid (trilinear)
  int64_t acqtab_off; // float offset of the staged acquisition table [N][12] in the workspace
  int32_t V, N, K, C, P;
  int32_t mode, bias, n_bias, learn_d, nbh, priors;
  int32_t ntab;       // neighbour-table entries (nbh, or 6 for the bias TV alone)
  int32_t nx, ny, nz;
  float bsc[3], boff[3]; // quadratic bias coordinates xi_a = i_a bsc[a] + boff[a] in [-1, 1]
                         // (2/(n_a - 1) and -1; both 0 when n_a = 1)
  int32_t acq_off;    // offset of the group's measurements in the acquisition arrays
  int32_t nb0;        // measurements with b = 0 at the start of the acquisition
  int32_t rec_stride; // float64 fields per record
  int32_t item_begin, item_count;
  int32_t tile_begin, tile_count;  // first-stage reduction tiles of this group
  float invM;         // 1/|M| (0 when the group is empty)
  // per-group float constants of the fused pass, formed once on the host (the
  // device has no scalar float unit: formed in the kernel they would sit in
  // vector registers across the measurement loop)
  float sdata;        // scale of the data term's seed: 2/|M| (MSE) or 1 (NLL)
  float sc_sp, sc_rep, sc_spa, sc_orph, sc_ord, sc_tv;  // prior weights lam/|M|
  float sc_cont2;     // -2 lam_cont / |M|
  float inv_s0o;      // 1 / s0_orphan
  float sc_orph_s0;   // lam_orphan / |M| / s0_orphan
  float tri_sc[3];    // 7 / (n_a - 1): trilinear control-grid coordinate per voxel step (0 if n_a = 1)
};

struct ItemDev {
  int32_t group;
  int32_t v0;       // first voxel (group-local)
  int32_t nv;       // voxels
  int32_t rec;      // record index within the group
  int32_t n_split;  // waves sharing one voxel row of the block (1, 2 or 4)
  int32_t kind;     // kernel variant ((K-1)*2 + mode)*2 + learned-D, for the persistent launch
};

// first-stage reduction tile: records [r0, r0+nr) of one group, fields [f0, f0+nf)
struct TileDev {
  int32_t group, r0, nr, f0, nf, out;  // out: float64 offset of the tile's partial row
};

struct ModelDev {
  float d_csf, d_gm, d_res, d_par, d_perp;
  float lam_sp, huber_delta, lam_rep, lam_sparse, tau_sparse;
  float lam_alpha, lam_beta, lam_bias;
  float lam_orphan, s0_orphan, lam_cont, lam_order, lam_tv;
};

struct PassArgs {
  const GroupDev* groups;
  const ItemDev* items;
  const float* bval;
  const float* bvec;
  const int32_t* coords;   // packed i | j << 10 | k << 20
  const int32_t* nbr;
  const float* ninv;       // 1/|N(x)| per voxel
  const float* y;
  const float* th_micro;
  const float* th_cal;
  float* g_micro;
  double* rec;
  float* wsp;              // workspace floats (spatial weights, per-voxel dlogB, acquisition tables)
  uint32_t* status;
  ModelDev model;
  int32_t item_base;       // first item of this launch
  int32_t n_items;         // items in this launch
  int32_t n_split;         // cross-wave buffer rows of the launch (max over items of rows*(WN-1))
  int32_t synth_only;      // forward model only (yhat written to g_micro as float [N][V])
  float* yhat;
  // fused Adam (adam != 0): the epilogue updates theta_micro (th_upd, the same buffer as
  // th_micro), m_micro and v_micro in place instead of storing the gradient
  int32_t adam;
  float* th_upd;
  float* m_micro;
  float* v_micro;
  const int32_t* step;
  float lr, b1, b2, eps;
  // set by prism_iteration_adam when the step counter advances at the start of
  // the call (k_fractions, block 0): the Adam updates then use t = step[0]
  int32_t* step_advance;   // the counter to advance (nullptr: no advance here)
  int32_t step_ready;      // 1: step[0] already counts this step
  double* calsq;           // [n_groups][3] sums of squares of alpha, beta, bias (nullptr: not needed)
  int32_t n_groups;
};

struct ReduceArgs {
  const GroupDev* groups;
  const TileDev* tiles;
  const double* rec;
  double* part;            // first-stage partial rows
  const float* th_cal;
  float* g_cal;
  double* loss;
  const float* wsp;
  const int32_t* grid;
  const int32_t* coords;
  uint32_t* status;
  ModelDev model;
  int32_t n_tiles;
  int32_t n_groups;
  // calibration Adam applied where each gradient entry is written (fused
  // iteration): theta_cal, moments and hyper-parameters; t = step[0]
  int32_t cal_adam;
  float* th_cal_upd;       // the same buffer as th_cal
  float* m_cal;
  float* v_cal;
  const int32_t* step;
  float lr, b1, b2, eps;
  const double* calsq;     // precomputed [n_groups][3] (the cal prior's loss) or nullptr
  // loss-history ring [hist_len][n_groups][terms] (or nullptr): the loss rows also go
  // to slot (hist_step[0] - hist_adv) mod hist_len, the iteration's index
  double* hist;
  const int32_t* hist_step;
  int32_t hist_len, hist_adv;
};

struct StitchArgs {
  const GroupDev* groups;
  const int32_t* src_g;    // [2][n_out] source group (-1: none)
  const int32_t* src_v;    // [2][n_out] source voxel within the group
  const float* src_w;      // [2][n_out] normalised blend weight
  const float* th_micro;
  float* maps;             // [P][n_out]
  int64_t n_out;
};

// launchers (prism_kernels.hip)
// spatial_c: the C shared by every group with the Eq. 7 prior (0: none, or they differ)
// max_nv: voxels of the largest work item
hipError_t launch_spatial(const PassArgs& a, int n_items, int spatial_c, int max_nv, hipStream_t s);
hipError_t launch_stage(const PassArgs& a, int n_groups, hipStream_t s);
// persistent launch of one register class (persistent_class(K) of its items)
int persistent_class(int K);
hipError_t launch_pass_persistent(const PassArgs& a, int cls, int maxN, int grid, int32_t* counter,
                                  hipStream_t s);
int persistent_blocks_per_cu(int cls, int maxN, int xsplit);
// launch facts of the fused pass's per-variant kernels: LDS bytes per block (static
// and dynamic) and the waves per SIMD its register budget allows
size_t pass_lds_per_block(int maxN, int xsplit, int K, int learn_d, int vpl);
int pass_waves_per_simd(int K, int mode, int learn_d, int vpl);
// every fused-pass variant of one K (one translation unit per K)
template <int K>
hipError_t launch_pass_k(const PassArgs& a, int mode, int learn_d, int vpl, int maxN, hipStream_t s);
hipError_t launch_pass_maxn(const PassArgs& a, int K, int mode, int learn_d, int vpl, int maxN,
                            hipStream_t s);
hipError_t launch_reduce(const ReduceArgs& a, int max_tile_fields, hipStream_t s);
hipError_t launch_bias_trilinear(const ReduceArgs& a, const int32_t* tri_groups, int n_tri,
                                 hipStream_t s);
hipError_t launch_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr,
                       float b1, float b2, float eps, int32_t* step, hipStream_t s,
                       bool advance = true);
hipError_t launch_stitch(const StitchArgs& a, int K, int learn_d, hipStream_t s);
hipError_t launch_rprop(float* p, const float* g, float* prev, float* step, int64_t n,
                        float em, float ep, float smin, float smax, hipStream_t s);

hipError_t launch_rician_terms(const float* z, float* li, float* omr, float* q, int64_t n, hipStream_t s);

// Static device workspace of prism_loss_grad_noalloc (prism_kernels.hip): its
// size, the per-device set-up (hipGetSymbolAddress with `device` current, once
// per device) and the address found by that set-up (nullptr and the error if
// it failed or has not run).
constexpr size_t kStaticScratchBytes = (size_t)64 << 20;
hipError_t static_scratch_setup(int device);
void* static_scratch(int device, hipError_t* err);

}  // namespace prism
