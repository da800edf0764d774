// The fused forward + adjoint pass (k_pass) and the forward model (k_synth)
// as templates over (K, data mode, learned diffusivities, voxels per lane).
// Each K is instantiated in its own translation unit (prism_pass_k.hip
// compiled with PRISM_PASS_K = 1..6) and the persistent launch inlines every
// variant (prism_persistent.hip).
#pragma once
#include <algorithm>

#include "prism_common.h"

namespace prism {

#ifndef PRISM_PASS_MIN_WAVES
#define PRISM_PASS_MIN_WAVES 1
#endif
#ifndef PRISM_PERSISTENT_MIN_WAVES
#define PRISM_PERSISTENT_MIN_WAVES 2
#endif
#ifndef PRISM_PREFETCH
#define PRISM_PREFETCH 4
#endif
#ifndef PRISM_FOUR_WAVES
#define PRISM_FOUR_WAVES 1
#endif
// measurements per tile of the per-measurement sums (one per lane of a row of 16)
constexpr int kTile = 16;
// depth of the y prefetch ring (measurements ahead); kTile is a multiple of it
constexpr int kPf = PRISM_PREFETCH;
static_assert(kTile % kPf == 0, "tile must be a multiple of the prefetch depth");


// Waves per SIMD that the register allocation of the fused pass must allow.
// MSE with fixed diffusivities and at most three fibres, one voxel per lane:
// four (128 registers; the measurement loop stays free of spills, the few
// spills are in the per-voxel prologue and epilogue), scheduling one
// measurement at a time.  Otherwise three for the variants that fit 168
// registers without spilling (one voxel per lane, at most two fibres, or three
// with fixed diffusivities), letting the scheduler interleave two measurements
// at a time (sched_span 2); else PRISM_PASS_MIN_WAVES, one measurement at a time.
constexpr bool pass_four_waves(int K, int MODE, bool LD, int VL) {
  return PRISM_FOUR_WAVES && VL == 1 && MODE == 0 && !LD && K <= 3;
}
constexpr int pass_min_waves(int K, int MODE, bool LD, int VL) {
  return pass_four_waves(K, MODE, LD, VL) ? 4
         : VL == 1 && (K <= 2 || (K == 3 && !LD)) ? 3 : PRISM_PASS_MIN_WAVES;
}
constexpr int sched_span(int K, int MODE, bool LD, int VL) {
  return pass_min_waves(K, MODE, LD, VL) == 3 ? 2 : 1;
}

// ---------------------------------------------------------------------------
// staging of one measurement: 3 x float4.  With fixed diffusivities:
//   a = (s gx, s gy, s gz, kpar)   s = sqrt(b Dpar log2(e)), kpar = -b Dpar log2(e)
//   b = (kperp, Ecsf, Egm, Eres)   kperp = -b Dperp log2(e); the balls' Eq. 4
//   c = (exp(alpha_n), beta_n, Dperp/Dpar - 1, 0)
// so that with cs = (s g).d = s cos the fibre terms are e1 = exp2(-cs^2) and
// e12 = exp2(kperp + (Dperp/Dpar - 1) cs^2), and d cs / d d = s g is the
// staged vector itself.  With learned diffusivities (Dpar, Dperp per voxel):
//   a = (gx, gy, gz, -b log2(e)), b = (-b log2(e), Ecsf, Egm, Eres),
//   c = (exp(alpha_n), beta_n, -2 b, 0)
// (the fourth component of a and of c is not read with fixed diffusivities: the
// three read share one LDS load)
// ---------------------------------------------------------------------------
inline __device__ void stage_acquisition(const PassArgs& A, const GroupDev& g, float4* acq) {
  const float* cal = A.th_cal + g.cal_off;
  const float* alpha = cal + g.n_bias;
  const float* beta = alpha + g.N;
  const float dpar = g.learn_d ? 1.0f : A.model.d_par;     // d_par > 0 (checked at create)
  const float dperp = g.learn_d ? 1.0f : A.model.d_perp;
  for (int n = threadIdx.x; n < g.N; n += blockDim.x) {
    const float b = A.bval[g.acq_off + n];
    const float* gv = A.bvec + 3 * (int64_t)(g.acq_off + n);
    const float kpar = -b * dpar * kLog2e, kperp = -b * dperp * kLog2e;
    const float s = g.learn_d ? 1.0f : sqrtf(-kpar);
    acq[3 * n + 0] = make_float4(s * gv[0], s * gv[1], s * gv[2], kpar);
    acq[3 * n + 1] = make_float4(kperp, expf(-b * A.model.d_csf), expf(-b * A.model.d_gm),
                                 expf(-b * A.model.d_res));
    acq[3 * n + 2] = make_float4(expf(alpha[n]), beta[n], g.learn_d ? -2.0f * b : dperp / dpar - 1.0f, 0.0f);
  }
}

// ---------------------------------------------------------------------------
// per-voxel state
// ---------------------------------------------------------------------------
// A fibre's attenuation (Eq. 5) is E_k = f_in e1 + (1 - f_in) e12 with
// e1 = exp(-b Dpar cos^2) and e12 = e1 e2 = exp(-b Dpar cos^2 - b Dperp sin^2):
// both are taken as one exp each, so e2 itself is never formed, and every
// per-voxel factor (B S0 f_k f_in, B S0 f_k (1 - f_in)) multiplies them directly.
template <int K, bool LD>
struct Vox {
  float Fi[3];      // B S0 * fraction of csf, gm, res (bias field folded in)
  float Fa[K];      // B S0 f_k f_in:       weight of e1
  float Fb[K];      // B S0 f_k (1 - f_in): weight of e12
  float d[K][3];    // unit directions
  float a1, a2;     // learned D: Dpar f_in, (Dpar - Dperp)(1 - f_in), dE/dcos = -2b cos (a1 e1 + a2 e12);
                    // fixed D: -2 ln2 f_in, -2 ln2 (1 - Dperp/Dpar)(1 - f_in), dE/dcs = cs (a1 e1 + a2 e12)
  float dpar, dperp;
};

// per-voxel adjoint accumulators as one register array (constant indices only);
// with dS = seed exp(alpha_n) the sums over the measurements are
//   r[0..2]        sum dS E_c  of csf, gm, res
//   r[kE1 + k]     sum dS e1_k,  r[kE12 + k] sum dS e12_k
//                  (fibre k's sum dS E_k = f_in r[kE1+k] + (1 - f_in) r[kE12+k] and
//                  its f_in derivative sum dS (e1 - e12) come from these per voxel)
//   r[kGd + 3k..]  sum dcos_k g_n, the direction adjoint divided by F_k
// and the log-bias adjoint sum seed (yhat - beta) = sum_c F_c sum dS E_c is
// formed from them per voxel.
template <int K, bool LD>
struct Acc {
  static constexpr int kE1 = 3;
  static constexpr int kE12 = 3 + K;
  static constexpr int kGd = 3 + 2 * K;
  static constexpr int kDpar = 3 + 5 * K;     // learned diffusivities
  static constexpr int kDperp = 4 + 5 * K;
  static constexpr int N = 3 + 5 * K + (LD ? 2 : 0);
  float r[N];
};
constexpr int acc_count(int K, bool LD) { return 3 + 5 * K + (LD ? 2 : 0); }


struct Derived {            // quantities the epilogue needs again
  float S0, sig_s;
  float f[kMaxC];
  float invn[kMaxK];
  float fin, omf;           // f_intra, 1 - f_intra
  float sig_dpar, sig_dperp;
  float B;                  // bias field
};

__device__ __forceinline__ float log_bias(const GroupDev& g, const float* cal, int32_t pc) {
  if (g.bias == 0) return 0.0f;
  const int i = pc & 1023, j = (pc >> 10) & 1023, k = (pc >> 20) & 1023;
  if (g.bias == 1) {
    // xi_a = (2 i_a - (n_a - 1)) / (n_a - 1) as one FMA with per-group constants
    const float x = fmaf((float)i, g.bsc[0], g.boff[0]);
    const float y = fmaf((float)j, g.bsc[1], g.boff[1]);
    const float z = fmaf((float)k, g.bsc[2], g.boff[2]);
    float s = cal[0];
    s = fmaf(cal[1], x, s);
    s = fmaf(cal[2], y, s);
    s = fmaf(cal[3], z, s);
    s = fmaf(cal[4], x * x, s);
    s = fmaf(cal[5], y * y, s);
    s = fmaf(cal[6], z * z, s);
    s = fmaf(cal[7], x * y, s);
    s = fmaf(cal[8], x * z, s);
    s = fmaf(cal[9], y * z, s);
    return s;
  }
  // trilinear 8^3: control point c sits at voxel c (n-1)/7 along each axis
  float p[3];
  int i0[3];
  const int ii[3] = {i, j, k};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float pa = ii[a] * g.tri_sc[a];
    int c = (int)floorf(pa);
    c = c > 6 ? 6 : c;
    i0[a] = c;
    p[a] = pa - c;
  }
  float s = 0.0f;
#pragma unroll
  for (int cx = 0; cx < 2; ++cx)
#pragma unroll
    for (int cy = 0; cy < 2; ++cy)
#pragma unroll
      for (int cz = 0; cz < 2; ++cz) {
        const float w = (cx ? p[0] : 1.0f - p[0]) * (cy ? p[1] : 1.0f - p[1]) *
                        (cz ? p[2] : 1.0f - p[2]);
        s = fmaf(w, cal[((i0[0] + cx) * 8 + (i0[1] + cy)) * 8 + (i0[2] + cz)], s);
      }
  return s;
}

// Raw parameters of voxel v -> constrained quantities (Sec. 2.2, 2.5).  Called
// in the prologue (Vox for the measurement loop) and again in the epilogue
// (Derived for the chain rule), so that nothing but Vox stays live across the
// measurement loop.
template <int K, bool LD>
__device__ __forceinline__ void load_voxel(const PassArgs& A, const GroupDev& g, int v,
                                           Vox<K, LD>& x, Derived& dv, bool& zero_dir) {
  constexpr int C = K + 3;
  const float* th = A.th_micro + g.micro_off;
  const int64_t V = g.V;
  const uint32_t rowb = (uint32_t)V * 4u, off = (uint32_t)v * 4u;  // rows of V floats
  auto at = [&](int row) { return load_row_f32(row_base(th, row, V), rowb, off); };
  const float s = at(0);
  dv.S0 = softplus_f(s);
  dv.sig_s = sigmoid_f(s);
  float lg[C];
  float m = -INFINITY;
#pragma unroll
  for (int c = 0; c < C; ++c) {
    lg[c] = at(row_logit(c));
    m = fmaxf(m, lg[c]);
  }
  float sum = 0.0f;
#pragma unroll
  for (int c = 0; c < C; ++c) {
    lg[c] = exp_hw(lg[c] - m);
    sum += lg[c];
  }
  const float inv = rcp(sum);
  const float* cal = A.th_cal + g.cal_off;
  dv.B = exp_hw(log_bias(g, cal, A.coords[g.vox_off + v]));
  const float BS0 = dv.B * dv.S0;
#pragma unroll
  for (int c = 0; c < C; ++c) dv.f[c] = lg[c] * inv;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const float vx = at(row_v(C, k, 0));
    const float vy = at(row_v(C, k, 1));
    const float vz = at(row_v(C, k, 2));
    const float n2 = fmaf(vx, vx, fmaf(vy, vy, vz * vz));
    float in = 0.0f;
    if (n2 > 0.0f) {
      in = rsq(n2);
    } else {
      zero_dir = true;
    }
    dv.invn[k] = in;
    x.d[k][0] = vx * in;
    x.d[k][1] = vy * in;
    x.d[k][2] = vz * in;
  }
  const float fin = sigmoid_f(at(row_fin(C, K)));
  const float omf = 1.0f - fin;
  dv.fin = fin;
  dv.omf = omf;
  x.Fi[0] = BS0 * dv.f[0];
  x.Fi[1] = BS0 * dv.f[1];
  x.Fi[2] = BS0 * dv.f[C - 1];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const float F = BS0 * dv.f[2 + k];
    x.Fa[k] = F * fin;
    x.Fb[k] = F * omf;
  }
  if (LD) {
    const float a = at(row_dpar(C, K));
    const float b = at(row_dpar(C, K) + 1);
    x.dpar = softplus_f(a);
    x.dperp = softplus_f(b);
    dv.sig_dpar = sigmoid_f(a);
    dv.sig_dperp = sigmoid_f(b);
  } else {
    x.dpar = 0.0f;
    x.dperp = 0.0f;
    dv.sig_dpar = 0.0f;
    dv.sig_dperp = 0.0f;
  }
  if (LD) {
    x.a1 = x.dpar * fin;
    x.a2 = (x.dpar - x.dperp) * omf;
  } else {
    // d E / d cs = -2 ln 2 cs (f_in e1 + (1 - Dperp/Dpar)(1 - f_in) e12)
    x.a1 = -2.0f * kLn2 * fin;
    x.a2 = -2.0f * kLn2 * (1.0f - A.model.d_perp / A.model.d_par) * omf;
  }
}

// ---------------------------------------------------------------------------
// one (voxel, measurement) pair: forward, data term, adjoint accumulation
// ---------------------------------------------------------------------------
// Data term of one pair (Eq. 8 / Eq. 9) at yhat = gain S + beta (Eq. 6) and its
// seed dL/dyhat (MSE: without the 2/|M| applied per voxel later).  valid (0 for
// lanes past the end of the item) zeroes the lane's residual, so the loss, the
// per-measurement sums and the (unstored) adjoint all drop it.
template <int MODE>
__device__ __forceinline__ void data_term(float S, float gain, float beta, float yv, float valid,
                                          float inv_s2, float& t_loss, float& t_sig, float& seed) {
  if (MODE == kMSE) {
    const float r = fmaf(gain, S, beta - yv) * valid;
    seed = r;
    t_loss = r * r;
    t_sig = 0.0f;
  } else {
    const float yh = fmaf(gain, S, beta);
    const float ay = fabsf(yv), ah = fabsf(yh);
    const float z = ay * ah * inv_s2;
    float omr, qz;
    const float li = log_i0e(z, omr, qz);
    const float dd = ah - ay;
    t_loss = fmaf(dd * dd, 0.5f * inv_s2, -li) * valid;
    t_sig = fmaf(dd * dd, inv_s2, qz) * valid;  // qz = 2z (1 - R(z))
    const float sd = fmaf(ay, omr, dd) * inv_s2 * valid;
    seed = yh < 0.0f ? -sd : sd;          // sgn(yhat) [(|yhat|-|y|) + |y|(1-R)] / s^2
  }
}

// One pair at b = 0: every attenuation of Eq. 4-5 is exactly 1, so S = sum_c F_c
// (Fsum) and the fibre-angle, f_intra and diffusivity adjoints vanish; the
// compartments' adjoint, dS for each of them, is summed once (dS0) and added to
// every compartment after the b = 0 measurements.  sq = seed S: the
// per-measurement sum of sq times exp(alpha_n) is the alpha_n adjoint.
template <int MODE>
__device__ __forceinline__ void pair_b0(float Fsum, float& dS0, float yv, float valid, const float4 c,
                                        float inv_s2, float& t_loss, float& t_sig, float& sq, float& seed) {
  data_term<MODE>(Fsum, c.x, c.y, yv, valid, inv_s2, t_loss, t_sig, seed);
  sq = seed * Fsum;
  dS0 = fmaf(seed, c.x, dS0);
}

template <int K, int MODE, bool LD>
__device__ __forceinline__ void pair(const Vox<K, LD>& x, Acc<K, LD>& acc, float yv, float valid,
                                     const float4 a, const float4 b, const float4 c, float inv_s2,
                                     float& t_loss, float& t_sig, float& sq, float& seed) {
  using AC = Acc<K, LD>;
  // fixed D: (gx, gy, gz) = s g and cc = s cos (see stage_acquisition)
  const float gx = a.x, gy = a.y, gz = a.z;
  const float kp = LD ? a.w * x.dpar : 0.0f;    // learned D: log2 e1 = kp cos^2
  const float kq = LD ? b.x * x.dperp : b.x;    // log2 e12 = kq + kd cc^2
  const float kd = LD ? kp - kq : c.z;
  float S = x.Fi[0] * b.y;
  S = fmaf(x.Fi[1], b.z, S);
  S = fmaf(x.Fi[2], b.w, S);
  float cc[K], e1[K], e12[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    cc[k] = fmaf(gz, x.d[k][2], fmaf(gy, x.d[k][1], gx * x.d[k][0]));
    const float c2 = cc[k] * cc[k];
    e1[k] = ex2(LD ? kp * c2 : -c2);      // exp(-b Dpar cos^2)
    e12[k] = ex2(fmaf(kd, c2, kq));       // exp(-b Dpar cos^2 - b Dperp sin^2)
    S = fmaf(x.Fa[k], e1[k], S);          // Eq. 3 with Eq. 5: F_k (f_in e1 + (1 - f_in) e12)
    S = fmaf(x.Fb[k], e12[k], S);
  }
  data_term<MODE>(S, c.x, c.y, yv, valid, inv_s2, t_loss, t_sig, seed);
  sq = seed * S;
  // dS = dL/dS / B: the F_c carry B, so dS F_c is the adjoint of compartment c's signal
  const float dS = seed * c.x;
  // the factor of the direction adjoint shared by the fibres: dS (-2b) (learned D),
  // dS (fixed D: -2 ln2 is in a1, a2 and the scale s in cc and the staged vector)
  const float dSz = LD ? dS * c.z : dS;
  // from three fibres on, fold dSz into the two per-voxel factors once per pair
  // (two products) rather than into each fibre's cosine (one product per fibre)
  constexpr bool kFold = K >= 3;
  const float a1z = kFold ? x.a1 * dSz : x.a1, a2z = kFold ? x.a2 * dSz : x.a2;
  acc.r[0] = fmaf(dS, b.y, acc.r[0]);
  acc.r[1] = fmaf(dS, b.z, acc.r[1]);
  acc.r[2] = fmaf(dS, b.w, acc.r[2]);
#pragma unroll
  for (int k = 0; k < K; ++k) {
    acc.r[AC::kE1 + k] = fmaf(dS, e1[k], acc.r[AC::kE1 + k]);
    acc.r[AC::kE12 + k] = fmaf(dS, e12[k], acc.r[AC::kE12 + k]);
    // dE/dcos = -2b cos (Dpar f_in e1 + (Dpar - Dperp)(1 - f_in) e12), here times dS
    // (fixed D: dE/dcs against the staged s g, the same product); the fibre's F_k
    // multiplies the sums once per voxel, after the loop
    const float dc = (kFold ? cc[k] : cc[k] * dSz) * fmaf(a1z, e1[k], a2z * e12[k]);
    acc.r[AC::kGd + 3 * k + 0] = fmaf(dc, gx, acc.r[AC::kGd + 3 * k + 0]);
    acc.r[AC::kGd + 3 * k + 1] = fmaf(dc, gy, acc.r[AC::kGd + 3 * k + 1]);
    acc.r[AC::kGd + 3 * k + 2] = fmaf(dc, gz, acc.r[AC::kGd + 3 * k + 2]);
    if (LD) {
      // dE/dDpar = -b cos^2 E, dE/dDperp = -b sin^2 (1-fin) e12, with -b = (-2b)/2
      const float mb = 0.5f * c.z;
      const float c2 = cc[k] * cc[k];
      const float FE = fmaf(x.Fa[k], e1[k], x.Fb[k] * e12[k]);
      acc.r[AC::kDpar] = fmaf(dS * FE, mb * c2, acc.r[AC::kDpar]);
      acc.r[AC::kDperp] = fmaf(dS * (x.Fb[k] * e12[k]), mb - mb * c2, acc.r[AC::kDperp]);
    }
  }
}

static_assert(kPf == 4, "the per-measurement sums take four measurements at a time");

// Measurements [nb, ne) for the VL voxels of this lane, in tiles of kTile.
// The per-measurement sums over the wave's 64 x VL voxels (the beta_n adjoint,
// and the alpha_n adjoint divided by exp(alpha_n), which multiplies the tile's
// totals) are reduced over each row of 16 lanes as the measurements arrive
// (RowScatter, four at a time); after the tile lane l holds its row's sum for
// measurement n0 + row_scatter_index(l), and two lane exchanges (xor 16,
// xor 32) add the four rows.  Invalid lanes (beyond the item) carry valid = 0,
// which removes them from every sum.  FULL: every lane's voxels are in the
// item (the validity factors are 1 and drop out at compile time).
template <int K, int MODE, bool LD, int VL, bool FULL>
__device__ __forceinline__ void measurement_loop(const Vox<K, LD> (&x)[VL], Acc<K, LD> (&acc)[VL],
                                                 const float* yg, int64_t V, const int (&vox)[VL],
                                                 const float (&valid)[VL],
                                                 const float4* __restrict__ acq,
                                                 int nb, int ne, int nb0, int N, float inv_s2, int lane,
                                                 float* wacc, double& dloss, double& dsig) {
  uint32_t voff[VL];  // byte offsets of the lane's voxels in a row of y
#pragma unroll
  for (int j = 0; j < VL; ++j) voff[j] = (uint32_t)vox[j] * 4u;
  const uint32_t rowb = (uint32_t)V * 4u;  // bytes in a row of y (V <= 1023^3)
  // y prefetch ring kPf measurements deep (slot u holds measurement nb + u mod kPf)
  float yr[kPf][VL];
#pragma unroll
  for (int u = 0; u < kPf; ++u)
#pragma unroll
    for (int j = 0; j < VL; ++j) yr[u][j] = load_row_f32(yg + (int64_t)min(nb + u, ne - 1) * V, rowb, voff[j]);
  const RowScatterMasks sm = row_scatter_masks(lane);
  const int bank = (lane >> 2) & 3;   // the group of four measurements this lane's row sums keep
  RowScatter sa, sb;                  // the alpha and beta sums of the tile
  float lacc, sacc;
  int n0 = nb;
  // one measurement, u = n - n0 mod 4: the ring slot u is refilled (measurement
  // n + kPf) only after its value has been consumed, so the load can target the
  // slot's register directly and the wait for it lands kPf measurements later
  auto body = [&](int t, int u, float (&slot)[VL]) {
    const int n = n0 + t;
    const float4 a = acq[3 * n + 0];
    const float4 b = acq[3 * n + 1];
    const float4 c = acq[3 * n + 2];
    float pa = 0.0f, pb = 0.0f;
#pragma unroll
    for (int j = 0; j < VL; ++j) {
      float tl, ts, sq, sd;
      pair<K, MODE, LD>(x[j], acc[j], slot[j], FULL ? 1.0f : valid[j], a, b, c, inv_s2, tl, ts, sq, sd);
      lacc += tl;
      if (MODE == kNLL) sacc += ts;
      pa = j == 0 ? sq : pa + sq;
      pb = j == 0 ? sd : pb + sd;
    }
    // refill from the measurement's row (a uniform base) at the lane's voxel
    const float* row = yg + (int64_t)min(n + kPf, ne - 1) * V;  // clamped: in bounds
#pragma unroll
    for (int j = 0; j < VL; ++j) slot[j] = load_row_f32(row, rowb, voff[j]);
    row_scatter_push(sa, pa, u, sm);
    row_scatter_push(sb, pb, u, sm);
  };
  // a measurement past the end of the range: zeros complete the group
  auto body_none = [&](int u) {
    row_scatter_push(sa, 0.0f, u, sm);
    row_scatter_push(sb, 0.0f, u, sm);
  };
  auto group_end = [&](int t0) {
    const bool here = bank == (t0 >> 2);
    row_scatter_group(sa, here);
    row_scatter_group(sb, here);
  };
  auto tile_begin = [&]() {
    lacc = 0.0f;
    sacc = 0.0f;
    sa.acc = 0.0f;
    sb.acc = 0.0f;
  };
  // the same at b = 0 (see pair_b0)
  float Fsum[VL], dS0[VL];
  auto body_b0 = [&](int t, int u, float (&slot)[VL]) {
    const int n = n0 + t;
    const float4 c = acq[3 * n + 2];
    float pa = 0.0f, pb = 0.0f;
#pragma unroll
    for (int j = 0; j < VL; ++j) {
      float tl, ts, sq, sd;
      pair_b0<MODE>(Fsum[j], dS0[j], slot[j], FULL ? 1.0f : valid[j], c, inv_s2, tl, ts, sq, sd);
      lacc += tl;
      if (MODE == kNLL) sacc += ts;
      pa = j == 0 ? sq : pa + sq;
      pb = j == 0 ? sd : pb + sd;
    }
    const float* row = yg + (int64_t)min(n + kPf, ne - 1) * V;  // clamped: in bounds
#pragma unroll
    for (int j = 0; j < VL; ++j) slot[j] = load_row_f32(row, rowb, voff[j]);
    row_scatter_push(sa, pa, u, sm);
    row_scatter_push(sb, pb, u, sm);
  };
  // four straight-line measurements from t0 (a multiple of kPf)
  auto group = [&](int t0) {
#pragma unroll
    for (int u = 0; u < kPf; ++u) {
      body(t0 + u, u, yr[u]);
      if ((u + 1) % sched_span(K, MODE, LD, VL) == 0) __builtin_amdgcn_sched_barrier(0);
    }
    group_end(t0);
  };
  // wave totals of the tile's per-measurement sums (cnt measurements)
  auto tile_end = [&](int cnt) {
    float ra = sa.acc, rb = sb.acc;
    ra += xor16_f32(ra);
    rb += xor16_f32(rb);
    ra += xor32_f32(ra);
    rb += xor32_f32(rb);
    const int tn = row_scatter_index(lane);
    if (lane < kTile && tn < cnt) {
      const int n = n0 + tn;
      wacc[n] = fmaf(ra, acq[3 * n + 2].x, wacc[n]);  // times exp(alpha_n)
      wacc[N + n] += rb;
    }
    dloss += (double)lacc;
    if (MODE == kNLL) dsig += (double)sacc;  // 0 for MSE
  };
  // whole tiles of the acquisition's leading b = 0 measurements first
  const int b0end = min(nb0, ne);
  if (n0 + kTile <= b0end) {
#pragma unroll
    for (int j = 0; j < VL; ++j) {
      float sF = 0.0f;
#pragma unroll
      for (int cc = 0; cc < 3; ++cc) sF += x[j].Fi[cc];
#pragma unroll
      for (int k = 0; k < K; ++k) sF += x[j].Fa[k] + x[j].Fb[k];
      Fsum[j] = sF;
      dS0[j] = 0.0f;
    }
    for (; n0 + kTile <= b0end; n0 += kTile) {
      tile_begin();
#pragma unroll 1
      for (int t0 = 0; t0 < kTile; t0 += kPf) {
#pragma unroll
        for (int u = 0; u < kPf; ++u) body_b0(t0 + u, u, yr[u]);
        group_end(t0);
        __builtin_amdgcn_sched_barrier(0);
      }
      tile_end(kTile);
    }
#pragma unroll
    for (int j = 0; j < VL; ++j)
#pragma unroll
      for (int cc = 0; cc < 3 + 2 * K; ++cc) acc[j].r[cc] += dS0[j];  // e1 = e12 = 1
  }
  if (MODE == kMSE) {
    // whole tiles: every path into the loop has the ring's loads in flight in slot
    // order, so each wait is for exactly one slot
    for (; n0 + kTile <= ne; n0 += kTile) {
      tile_begin();
#pragma unroll 1
      for (int t0 = 0; t0 < kTile; t0 += kPf) group(t0);
      tile_end(kTile);
    }
    if (n0 < ne) {  // the range's last, partial tile
      const int cnt = ne - n0;
      const int full = cnt & ~(kPf - 1);  // cnt > 0
      tile_begin();
#pragma unroll 1
      for (int t0 = 0; t0 < full; t0 += kPf) group(t0);
      if (full < cnt) {
#pragma unroll
        for (int u = 0; u < kPf; ++u) {
          if (full + u < cnt)
            body(full + u, u, yr[u]);
          else
            body_none(u);
        }
        group_end(full);
      }
      tile_end(cnt);
    }
  } else {
    for (; n0 < ne; n0 += kTile) {
      const int cnt = min(kTile, ne - n0);
      tile_begin();
      for (int t0 = 0; t0 < cnt; t0 += kPf) {
#pragma unroll
        for (int u = 0; u < kPf; ++u) {
          if (t0 + u < cnt)
            body(t0 + u, u, yr[u]);
          else
            body_none(u);
        }
        group_end(t0);
      }
      tile_end(cnt);
    }
  }
}

// statically sized LDS of the fused pass (one instance per kernel, shared by the
// variants a persistent kernel inlines)
constexpr int kRecVals = 18;  // per-thread record values of the fused pass
struct PassShared {
  double wrec[4][kRecVals]; // per-wave record sums (the epilogue's terms added chunk by chunk)
  float adam_sc[2];         // fused Adam: step size and 1/sqrt(1 - b2^t)
};

// The fused pass over one work item (a run of one group's voxels).
template <int K, int MODE, bool LD, int VL>
__device__ __forceinline__ void pass_item(const PassArgs& A, const float4* __restrict__ acq_global,
                                          const ItemDev& it, float4* smem4, PassShared& sh) {
  auto& wrec = sh.wrec;
  constexpr int C = K + 3;
  constexpr int NACC = Acc<K, LD>::N;
  const GroupDev g = A.groups[it.group];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // wave-uniform (scalar)
  const int WN = it.n_split, rows = 4 / WN;
  const int row = wave / WN, split = wave - row * WN;
  const int N = g.N;
  float4* acq = smem4;                                       // [3N] unless read from SMEM
  float* accab = reinterpret_cast<float*>(smem4 + (PRISM_ACQ_SMEM ? 0 : 3 * N));  // [4][2][N]
  float* xbuf = accab + 8 * N;                               // [rows][WN-1][NACC][64*VL]

#if PRISM_ACQ_SMEM
  const float4* __restrict__ acq_tab = acq_global + g.acqtab_off / 4;
#else
  stage_acquisition(A, g, acq);
  const float4* acq_tab = acq;
#endif
  for (int i = tid; i < 8 * N; i += kBlock) accab[i] = 0.0f;
  if (lane < kRecVals) wrec[wave][lane] = 0.0;
  if (A.adam && tid == 0) adam_factors(A.step, A.lr, A.b1, A.b2, sh.adam_sc[0], sh.adam_sc[1], A.step_ready);
  __syncthreads();

  const int nb = (N * split) / WN, ne = (N * (split + 1)) / WN;
  const int64_t V = g.V;
  const float* yg = A.y + g.y_off;
  const float* cal = A.th_cal + g.cal_off;
  const float inv_s2 = MODE == kNLL ? expf(-2.0f * cal[g.n_bias + 2 * N]) : 0.0f;
  const float sdata = g.sdata;
  const bool has_sp = (g.priors & kPriorSpatial) && g.nbh > 0;
  float* wacc = accab + wave * 2 * N;

  double dloss = 0.0, dsig = 0.0;
  bool bad_grad = false, zero_dir = false;

  const int chunk = 64 * VL * rows;
  for (int cb = 0; cb < it.nv; cb += chunk) {
    int vox[VL];
    float valid[VL];
#pragma unroll
    for (int j = 0; j < VL; ++j) {
      const int lv = cb + row * 64 * VL + j * 64 + lane;
      const bool ok = lv < it.nv;
      valid[j] = ok ? 1.0f : 0.0f;
      vox[j] = it.v0 + (ok ? lv : 0);
    }
    Vox<K, LD> x[VL];
    Acc<K, LD> acc[VL];
#pragma unroll
    for (int j = 0; j < VL; ++j) {
      Derived dv_unused;
      load_voxel<K, LD>(A, g, vox[j], x[j], dv_unused, zero_dir);
#pragma unroll
      for (int i = 0; i < NACC; ++i) acc[j].r[i] = 0.0f;
    }

    // a chunk that lies wholly inside the item runs the loop without validity factors
    if (cb + chunk <= it.nv)
      measurement_loop<K, MODE, LD, VL, true>(x, acc, yg, V, vox, valid, acq_tab, nb, ne, g.nb0, N, inv_s2, lane,
                                              wacc, dloss, dsig);
    else
      measurement_loop<K, MODE, LD, VL, false>(x, acc, yg, V, vox, valid, acq_tab, nb, ne, g.nb0, N, inv_s2, lane,
                                               wacc, dloss, dsig);

    // combine the per-voxel accumulators of the waves that split this row over n
    if (WN > 1) {
      if (split > 0) {
#pragma unroll
        for (int j = 0; j < VL; ++j) {
          float* dst = xbuf + (((row * (WN - 1) + split - 1) * NACC) * 64 * VL) + j * 64 + lane;
#pragma unroll
          for (int i = 0; i < NACC; ++i) dst[i * 64 * VL] = acc[j].r[i];
        }
      }
      __syncthreads();
      if (split == 0) {
        for (int s = 1; s < WN; ++s) {
#pragma unroll
          for (int j = 0; j < VL; ++j) {
            const float* src = xbuf + (((row * (WN - 1) + s - 1) * NACC) * 64 * VL) + j * 64 + lane;
#pragma unroll
            for (int i = 0; i < NACC; ++i) acc[j].r[i] += src[i * 64 * VL];
          }
        }
      }
    }

    // epilogue: priors, chain rule to raw parameters, gradient store
    if (split == 0) {
      // the chunk's epilogue terms per thread, summed over the wave after the chunk
      // (so that nothing of them is live across the measurement loop)
      double e_rep = 0.0, e_spa = 0.0;
      float e_orph = 0.0f, e_cont = 0.0f, e_ord = 0.0f, e_tv = 0.0f;
      float e_b[10];
#pragma unroll
      for (int q = 0; q < 10; ++q) e_b[q] = 0.0f;
      float* gm = A.g_micro + g.micro_off;
      const float sc_rep = g.sc_rep;
      const float sc_spa = g.sc_spa;
      const float sc_sp = g.sc_sp;
#pragma unroll
      for (int j = 0; j < VL; ++j) {
        if (valid[j] == 0.0f) continue;
        const int v = vox[j];
        const uint32_t vrowb = (uint32_t)V * 4u, voff = (uint32_t)v * 4u;  // rows of V entries
        Derived D;
        {
          Vox<K, LD> x_again;
          bool zd = false;
          load_voxel<K, LD>(A, g, v, x_again, D, zd);
        }
        using AC = Acc<K, LD>;
        // sum_n dS E_c per compartment (fibres: f_in e1 + (1 - f_in) e12)
        float aE[C];
        aE[0] = acc[j].r[0];
        aE[1] = acc[j].r[1];
        aE[C - 1] = acc[j].r[2];
#pragma unroll
        for (int k = 0; k < K; ++k)
          aE[2 + k] = fmaf(D.fin, acc[j].r[AC::kE1 + k], D.omf * acc[j].r[AC::kE12 + k]);
        const float BS0 = D.B * D.S0;
        float gF[C], gf[C];
        float gS0 = 0.0f, slb = 0.0f;
        const float sB = sdata * D.B;
#pragma unroll
        for (int c = 0; c < C; ++c) {
          gF[c] = sB * aE[c];
          gf[c] = D.S0 * gF[c];
          gS0 = fmaf(D.f[c], gF[c], gS0);
          slb = fmaf(BS0 * D.f[c], aE[c], slb);   // sum_n seed (yhat - beta) = sum_c F_c sum dS E_c
        }
        float gd[K][3];
        float sfin = 0.0f;                          // sum_k F_k sum dS dE_k/df_in
#pragma unroll
        for (int k = 0; k < K; ++k) {
          const float Fk = BS0 * D.f[2 + k];
          const float sF = sdata * Fk;
#pragma unroll
          for (int a = 0; a < 3; ++a) gd[k][a] = sF * acc[j].r[AC::kGd + 3 * k + a];
          sfin = fmaf(Fk, acc[j].r[AC::kE1 + k] - acc[j].r[AC::kE12 + k], sfin);
        }
        if (has_sp) {
          // Eq. 7 adjoint: w(x)|N(x)| - sum_{u in N(x)} w(u), weight rows [V][C]
          const float* wrow = A.wsp + g.w_off;
          const int32_t* nbr = A.nbr + g.nbr_off;
          float sum[C];
#pragma unroll
          for (int c = 0; c < C; ++c) sum[c] = 0.0f;
          int cnt = 0;
          // six neighbours per round trip: their table entries, then their weight
          // rows (an absent neighbour reads this voxel's row with factor 0)
          constexpr int kNb = 6;
          for (int q0 = 0; q0 < g.nbh; q0 += kNb) {
            int u[kNb];
#pragma unroll
            for (int e = 0; e < kNb; ++e)
              u[e] = q0 + e < g.nbh ? load_row_i32(row_base(nbr, q0 + e, V), vrowb, voff) : -1;
            float t[kNb][C];
#pragma unroll
            for (int e = 0; e < kNb; ++e) load_row<C>(wrow, u[e] >= 0 ? u[e] : v, C, t[e]);
#pragma unroll
            for (int e = 0; e < kNb; ++e) {
              const float on = u[e] >= 0 ? 1.0f : 0.0f;
              cnt += u[e] >= 0 ? 1 : 0;
#pragma unroll
              for (int c = 0; c < C; ++c) sum[c] = fmaf(on, t[e][c], sum[c]);
            }
          }
          const float fc = (float)cnt;
          float own[C];
          load_row<C>(wrow, v, C, own);
#pragma unroll
          for (int c = 0; c < C; ++c) gf[c] = fmaf(sc_sp, fmaf(own[c], fc, -sum[c]), gf[c]);
        }
        if (g.priors & kPriorRep) {
          float lr = 0.0f;
#pragma unroll
          for (int i = 0; i < K; ++i)
#pragma unroll
            for (int k = i + 1; k < K; ++k) {
              const float dot = x[j].d[i][0] * x[j].d[k][0] + x[j].d[i][1] * x[j].d[k][1] +
                                x[j].d[i][2] * x[j].d[k][2];
              const float ad = fabsf(dot);
              const float sg = dot > 0.0f ? 1.0f : (dot < 0.0f ? -1.0f : 0.0f);
              const float fi = D.f[2 + i], fk = D.f[2 + k];
              lr = fmaf(fi * fk, ad, lr);
              gf[2 + i] = fmaf(sc_rep * fk, ad, gf[2 + i]);
              gf[2 + k] = fmaf(sc_rep * fi, ad, gf[2 + k]);
              const float w2 = sc_rep * fi * fk * sg;
#pragma unroll
              for (int a = 0; a < 3; ++a) {
                gd[i][a] = fmaf(w2, x[j].d[k][a], gd[i][a]);
                gd[k][a] = fmaf(w2, x[j].d[i][a], gd[k][a]);
              }
            }
          e_rep += (double)lr;
        }
        if (g.priors & kPriorSparse) {
          float ls = 0.0f;
#pragma unroll
          for (int k = 0; k < K; ++k) {
            const float fk = D.f[2 + k];
            if (fk < A.model.tau_sparse) {
              ls += fk;
              gf[2 + k] += sc_spa;
            }
          }
          e_spa += (double)ls;
        }
        if (g.priors & kPriorOrphan) {
          // WM fractions where S0 is near zero: hinge max(0, 1 - S0/s0) on S0
          const float s0o = A.model.s0_orphan;
          const float sc = g.sc_orph;
          const float h = fmaxf(0.0f, fmaf(-D.S0, g.inv_s0o, 1.0f));
          float wsum = 0.0f;
#pragma unroll
          for (int k = 0; k < K; ++k) {
            wsum += D.f[2 + k];
            gf[2 + k] = fmaf(sc, h, gf[2 + k]);
          }
          if (D.S0 < s0o) gS0 -= g.sc_orph_s0 * wsum;
          e_orph += h * wsum;
        }
        if (g.priors & kPriorOrder) {
          // fibre slots in descending order of fraction: hinge on each adjacent pair
          const float sc = g.sc_ord;
          float lo = 0.0f;
#pragma unroll
          for (int k = 0; k + 1 < K; ++k) {
            const float gap = D.f[3 + k] - D.f[2 + k];
            if (gap > 0.0f) {
              lo += gap;
              gf[3 + k] += sc;
              gf[2 + k] -= sc;
            }
          }
          e_ord += lo;
        }
        if ((g.priors & kPriorCont) && g.nbh > 0) {
          // slot-wise alignment with the neighbours' directions; the pair (x, u)
          // enters the sums of x and of u, weighted 1/|N(x)| and 1/|N(u)|
          const int32_t* nbr = A.nbr + g.nbr_off;
          const float* ninv = A.ninv + g.ninv_off;
          const float* th = A.th_micro + g.micro_off;
          const float sc2 = g.sc_cont2;
          const float ax = ninv[v];
          float lc = 0.0f;
          for (int q = 0; q < g.nbh; ++q) {
            const int u = nbr[(int64_t)q * V + v];
            if (u < 0) continue;
            const float w = sc2 * (ax + ninv[u]);
#pragma unroll
            for (int k = 0; k < K; ++k) {
              const float ux = th[(int64_t)row_v(C, k, 0) * V + u];
              const float uy = th[(int64_t)row_v(C, k, 1) * V + u];
              const float uz = th[(int64_t)row_v(C, k, 2) * V + u];
              const float n2 = fmaf(ux, ux, fmaf(uy, uy, uz * uz));
              const float in = n2 > 0.0f ? rsq(n2) : 0.0f;
              const float dx = ux * in, dy = uy * in, dz = uz * in;
              const float dot = x[j].d[k][0] * dx + x[j].d[k][1] * dy + x[j].d[k][2] * dz;
              lc = fmaf(ax, fmaf(-dot, dot, 1.0f), lc);
              const float wd = w * dot;
              gd[k][0] = fmaf(wd, dx, gd[k][0]);
              gd[k][1] = fmaf(wd, dy, gd[k][1]);
              gd[k][2] = fmaf(wd, dz, gd[k][2]);
            }
          }
          e_cont += lc;
        }
        // softmax chain rule
        float gsum = 0.0f;
#pragma unroll
        for (int c = 0; c < C; ++c) gsum = fmaf(D.f[c], gf[c], gsum);
        float gout[4 * kMaxK + 7];
        gout[0] = D.sig_s * gS0;
#pragma unroll
        for (int c = 0; c < C; ++c) gout[row_logit(c)] = D.f[c] * (gf[c] - gsum);
#pragma unroll
        for (int k = 0; k < K; ++k) {
          const float pr = gd[k][0] * x[j].d[k][0] + gd[k][1] * x[j].d[k][1] + gd[k][2] * x[j].d[k][2];
#pragma unroll
          for (int a = 0; a < 3; ++a)
            gout[row_v(C, k, a)] = (gd[k][a] - pr * x[j].d[k][a]) * D.invn[k];
        }
        gout[row_fin(C, K)] = D.fin * D.omf * sdata * sfin;
        if (LD) {
          gout[row_dpar(C, K)] = D.sig_dpar * sdata * acc[j].r[Acc<K, LD>::kDpar];
          gout[row_dpar(C, K) + 1] = D.sig_dperp * sdata * acc[j].r[Acc<K, LD>::kDperp];
        }
        constexpr int P = 4 * K + 5 + (LD ? 2 : 0);
        if (A.adam) {
          // fused Adam on this voxel's parameters (only this thread touches them)
          const float ss = sh.adam_sc[0], ib = sh.adam_sc[1];
          float* th = A.th_upd + g.micro_off;
          float* mm = A.m_micro + g.micro_off;
          float* vv = A.v_micro + g.micro_off;
          // in two batches of parameters: each batch's loads are issued
          // together so that their latencies overlap, in few registers
          constexpr int kAdamBatch = (P + 1) / 2;
#pragma unroll
          for (int p0 = 0; p0 < P; p0 += kAdamBatch) {
            float pp[kAdamBatch], m1[kAdamBatch], v1[kAdamBatch];
#pragma unroll
            for (int q = 0; q < kAdamBatch; ++q)
              if (p0 + q < P) {
                pp[q] = load_row_f32(row_base(th, p0 + q, V), vrowb, voff);
                m1[q] = load_row_f32(row_base(mm, p0 + q, V), vrowb, voff);
                v1[q] = load_row_f32(row_base(vv, p0 + q, V), vrowb, voff);
              }
#pragma unroll
            for (int q = 0; q < kAdamBatch; ++q)
              if (p0 + q < P) {
                const int p = p0 + q;
                if (!isfinite(gout[p])) bad_grad = true;
                adam_one(pp[q], gout[p], m1[q], v1[q], A.b1, A.b2, A.eps, ss, ib);
                store_row_f32(row_base(th, p, V), vrowb, voff, pp[q]);
                store_row_f32(row_base(mm, p, V), vrowb, voff, m1[q]);
                store_row_f32(row_base(vv, p, V), vrowb, voff, v1[q]);
              }
            __builtin_amdgcn_sched_barrier(0);
          }
        } else {
#pragma unroll
          for (int p = 0; p < P; ++p) {
            if (!isfinite(gout[p])) bad_grad = true;
            store_row_f32(row_base(gm, p, V), vrowb, voff, gout[p]);
          }
        }
        // bias-field adjoint dL/dlogB(x)
        float glb = sdata * slb;
        if ((g.priors & kPriorTV) && g.bias != 0) {
          // |B(x+e_a) - B(x)| over the in-mask face pairs: x owns the pair toward +e_a
          // and takes the derivative of both pairs it belongs to
          const int32_t* nbr = A.nbr + g.nbr_off;
          const float* cal = A.th_cal + g.cal_off;
          const int32_t pc = A.coords[g.vox_off + v];
          const float lb0 = log_bias(g, cal, pc);
          const float B0 = D.B;
          float lt = 0.0f, gt = 0.0f;
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            const int32_t step = 1 << (10 * a);
            if (load_row_i32(row_base(nbr, 2 * a + 1, V), vrowb, voff) >= 0) {
              const float dl = log_bias(g, cal, pc + step) - lb0;
              lt = fmaf(B0, fabsf(expm1f(dl)), lt);
              gt += dl > 0.0f ? -B0 : (dl < 0.0f ? B0 : 0.0f);
            }
            if (load_row_i32(row_base(nbr, 2 * a, V), vrowb, voff) >= 0) {
              const float dl = lb0 - log_bias(g, cal, pc - step);
              gt += dl > 0.0f ? B0 : (dl < 0.0f ? -B0 : 0.0f);
            }
          }
          glb = fmaf(g.sc_tv, gt, glb);
          e_tv += lt;
        }
        if (g.bias == 1) {
          const int32_t pc = A.coords[g.vox_off + v];
          const int i = pc & 1023, jj = (pc >> 10) & 1023, k = (pc >> 20) & 1023;
          // the coordinates of log_bias, bit for bit
          const float xx = fmaf((float)i, g.bsc[0], g.boff[0]);
          const float yy = fmaf((float)jj, g.bsc[1], g.boff[1]);
          const float zz = fmaf((float)k, g.bsc[2], g.boff[2]);
          const float phi[10] = {1.0f, xx, yy, zz, xx * xx, yy * yy, zz * zz, xx * yy, xx * zz, yy * zz};
#pragma unroll
          for (int q = 0; q < 10; ++q) e_b[q] = fmaf(phi[q], glb, e_b[q]);
        } else if (g.bias == 2) {
          A.wsp[g.glb_off + v] = glb;
        }
      }
      // record fields 1-6 and 8-17 (the terms this group has), wave-uniform branches
      auto wadd = [&](int q, double x) {
        const double t = wave_sum_f64(x);
        if (lane == 0) wrec[wave][q] += t;
      };
      if (g.priors & kPriorRep) wadd(1, e_rep);
      if (g.priors & kPriorSparse) wadd(2, e_spa);
      if (g.priors & kPriorOrphan) wadd(3, (double)e_orph);
      if ((g.priors & kPriorCont) && g.nbh > 0) wadd(4, (double)e_cont);
      if (g.priors & kPriorOrder) wadd(5, (double)e_ord);
      if ((g.priors & kPriorTV) && g.bias != 0) wadd(6, (double)e_tv);
      if (g.bias == 1) {
#pragma unroll
        for (int q = 0; q < 10; ++q) wadd(8 + q, (double)e_b[q]);
      }
    }
    if (WN > 1) __syncthreads();  // xbuf is reused by the next chunk
  }

  // ---- item record: per-problem sums and per-measurement sums ----
  double* rec = A.rec + g.rec_off + (int64_t)it.rec * g.rec_stride;
  {
    const double sl = wave_sum_f64(dloss);
    const double ss = wave_sum_f64(dsig);
    if (lane == 0) {
      wrec[wave][0] = sl;
      wrec[wave][7] = ss;
    }
  }
  if (bad_grad) atomicOr(A.status, (uint32_t)kStNonfiniteGrad);
  if (zero_dir) atomicOr(A.status, (uint32_t)kStZeroDir);
  __syncthreads();
  if (tid < kRecVals) {
    const double s = wrec[0][tid] + wrec[1][tid] + wrec[2][tid] + wrec[3][tid];
    const int field = tid == 0 ? kRecData : tid == 1 ? kRecRep : tid == 2 ? kRecSparse
                      : tid < 7 ? kRecOrphan + (tid - 3) : tid == 7 ? kRecSigma
                      : kRecBias + (tid - 8);
    rec[field] = s;
  }
  for (int n = tid; n < N; n += kBlock) {
    rec[kRecAlpha + n] = (double)accab[n] + (double)accab[2 * N + n] + (double)accab[4 * N + n] +
                         (double)accab[6 * N + n];
    rec[kRecAlpha + N + n] = (double)accab[N + n] + (double)accab[3 * N + n] +
                             (double)accab[5 * N + n] + (double)accab[7 * N + n];
  }
}

// One block per item of one kernel variant.
template <int K, int MODE, bool LD, int VL>
__global__ __launch_bounds__(kBlock, pass_min_waves(K, MODE, LD, VL)) void k_pass(
    PassArgs A, const float4* __restrict__ acq_global) {
  extern __shared__ float4 smem4[];
  __shared__ PassShared sh;
  const ItemDev it = A.items[A.item_base + xcd_item(blockIdx.x, gridDim.x)];
  pass_item<K, MODE, LD, VL>(A, acq_global, it, smem4, sh);
}

// ---------------------------------------------------------------------------
// forward model only
// ---------------------------------------------------------------------------
template <int K, bool LD>
__global__ __launch_bounds__(kBlock) void k_synth(PassArgs A) {
  extern __shared__ float4 smem4[];
  const ItemDev it = A.items[A.item_base + blockIdx.x];
  const GroupDev g = A.groups[it.group];
  float4* acq = smem4;
  stage_acquisition(A, g, acq);
  __syncthreads();
  const int64_t V = g.V;
  float* out = A.yhat + g.y_off;
  bool zero_dir = false;
  for (int lv = threadIdx.x; lv < it.nv; lv += kBlock) {
    const int v = it.v0 + lv;
    Vox<K, LD> x;
    Derived dv;
    load_voxel<K, LD>(A, g, v, x, dv, zero_dir);
    for (int n = 0; n < g.N; ++n) {
      const float4 a = acq[3 * n], b = acq[3 * n + 1], c = acq[3 * n + 2];
      float S = x.Fi[0] * b.y;
      S = fmaf(x.Fi[1], b.z, S);
      S = fmaf(x.Fi[2], b.w, S);
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const float cc = fmaf(a.z, x.d[k][2], fmaf(a.y, x.d[k][1], a.x * x.d[k][0]));
        const float c2 = cc * cc;
        const float kp = LD ? a.w * x.dpar : 0.0f;
        const float kq = LD ? b.x * x.dperp : b.x;
        const float kd = LD ? kp - kq : c.z;
        S = fmaf(x.Fa[k], ex2(LD ? kp * c2 : -c2), S);
        S = fmaf(x.Fb[k], ex2(fmaf(kd, c2, kq)), S);
      }
      out[(int64_t)n * V + v] = fmaf(c.x, S, c.y);
    }
  }
  if (zero_dir && A.status) atomicOr(A.status, (uint32_t)kStZeroDir);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
// dynamic LDS: acquisition table, per-wave measurement sums and the cross-wave
// buffer of the worst measurement split in the launch (xsplit = max rows*(WN-1): 0, 2 or 3)
inline size_t pass_lds_bytes(int maxN, int xsplit, int nacc_, int vpl) {
  size_t b = (PRISM_ACQ_SMEM ? 0 : (size_t)maxN * 3 * sizeof(float4)) + (size_t)8 * maxN * sizeof(float);
  b += (size_t)xsplit * nacc_ * 64 * vpl * sizeof(float);
  return b;
}

template <int K, int MODE, bool LD, int VL>
static hipError_t launch_pass_t(const PassArgs& a, hipStream_t s, int maxN) {
  const size_t lds = pass_lds_bytes(maxN, a.n_split, acc_count(K, LD), VL);
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute((const void*)k_pass<K, MODE, LD, VL>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  if (a.synth_only) {
    hipLaunchKernelGGL((k_synth<K, LD>), dim3(a.n_items), dim3(kBlock),
                       (size_t)maxN * 3 * sizeof(float4), s, a);
  } else {
    hipLaunchKernelGGL((k_pass<K, MODE, LD, VL>), dim3(a.n_items), dim3(kBlock), lds, s, a,
                       reinterpret_cast<const float4*>(a.wsp));
  }
  return hipGetLastError();
}

// every variant of one K; explicitly instantiated per K in prism_pass_k.hip
template <int K>
hipError_t launch_pass_k(const PassArgs& a, int mode, int ld, int vpl, int maxN, hipStream_t s) {
  if (vpl == 2) {
    if (mode == kMSE) return ld ? launch_pass_t<K, kMSE, true, 2>(a, s, maxN) : launch_pass_t<K, kMSE, false, 2>(a, s, maxN);
    return ld ? launch_pass_t<K, kNLL, true, 2>(a, s, maxN) : launch_pass_t<K, kNLL, false, 2>(a, s, maxN);
  }
  if (mode == kMSE) return ld ? launch_pass_t<K, kMSE, true, 1>(a, s, maxN) : launch_pass_t<K, kMSE, false, 1>(a, s, maxN);
  return ld ? launch_pass_t<K, kNLL, true, 1>(a, s, maxN) : launch_pass_t<K, kNLL, false, 1>(a, s, maxN);
}

}  // namespace prism
