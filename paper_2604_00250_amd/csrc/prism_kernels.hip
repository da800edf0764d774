// HIP kernels of the PRISM analysis-by-synthesis pass for gfx950 (CDNA4, wave64)
// other than the fused pass itself (prism_pass.h, instantiated per K in
// prism_pass_k.hip, and its persistent form in prism_persistent.hip):
//
// k_fractions, k_spatial  Eq. 7: softmax fractions, then the residual weights
//             rho'(r)/|N| per voxel and compartment.
// k_reduce1/2 deterministic two-stage reduction of per-item records into the
//             calibration gradient and the loss terms.
// k_bias_tri  gradient of the 8^3 trilinear log-bias grid.
// k_stitch    blend of per-slab maps into whole-volume maps (slab fitting).
// k_adam, k_rprop  optimiser steps.
#include <algorithm>
#include <mutex>

#include "prism_common.h"

namespace prism {

// The two Eq. 7 kernels run one block per work item with up to kAuxBlock
// threads, one voxel per thread (the launch sizes the block to the largest
// item): with fewer threads each one walked several voxels and the dependent
// table-then-gather loads of each voxel in turn.
constexpr int kAuxBlock = 512;

// fractions f = softmax(logits) once per voxel, rows [V][C] (CT: see load_row)
// The first kernel of a call also does two small jobs of the fused iteration
// before anything reads or changes the parameters: block 0 advances the step
// counter, and blocks n_items.. (one per group) sum the squares of the group's
// calibration parameters for the calibration prior's loss.
template <int CT>
__global__ __launch_bounds__(kAuxBlock) void k_fractions(PassArgs A) {
  if (blockIdx.x == 0 && threadIdx.x == 0 && A.step_advance) {
    A.step_advance[0] = A.step_advance[0] + 1;
    A.step_advance[1] = 0;
  }
  if ((int)blockIdx.x >= A.n_items) {
    // one wave, fixed order (the same bits whatever the launch's block size)
    if (threadIdx.x >= 64) return;
    const int gi = blockIdx.x - A.n_items;
    const GroupDev g = A.groups[gi];
    const float* cal = A.th_cal + g.cal_off;
    double sa = 0.0, sb = 0.0, sw = 0.0;
    for (int i = threadIdx.x; i < g.n_bias; i += 64) sw += (double)cal[i] * cal[i];
    for (int i = threadIdx.x; i < g.N; i += 64) {
      sa += (double)cal[g.n_bias + i] * cal[g.n_bias + i];
      sb += (double)cal[g.n_bias + g.N + i] * cal[g.n_bias + g.N + i];
    }
    sa = wave_sum_f64(sa);
    sb = wave_sum_f64(sb);
    sw = wave_sum_f64(sw);
    if (threadIdx.x == 0) {
      A.calsq[3 * gi + 0] = sa;
      A.calsq[3 * gi + 1] = sb;
      A.calsq[3 * gi + 2] = sw;
    }
    return;
  }
  const ItemDev it = A.items[xcd_item(blockIdx.x, A.n_items)];
  const GroupDev g = A.groups[it.group];
  if (!((g.priors & kPriorSpatial) && g.nbh > 0)) return;
  const float* th = A.th_micro + g.micro_off;
  const int64_t V = g.V;
  const int C = CT ? CT : g.C;
  float* f_out = A.wsp + g.w_off + (int64_t)C * V;
  for (int lv = threadIdx.x; lv < it.nv; lv += blockDim.x) {
    const int v = it.v0 + lv;
    float f[kMaxC];
    softmax_at(th, V, C, v, f);
    float r[CT ? CT : kMaxC];
#pragma unroll
    for (int c = 0; c < (CT ? CT : kMaxC); ++c) r[c] = f[c];
    store_row<CT>(f_out, v, C, r);
  }
}

// Eq. 7 residual weights w_c(x) = rho'(r_c(x)) / |N(x)| from the stored fractions.
// Neighbours are taken six at a time: all six table entries are loaded, then
// all their fraction rows (an absent neighbour reads the voxel's own row with
// weight 0), so one round trip serves six neighbours.  CT is the launch's
// common C, or 0 when its groups differ in C.
template <int CT>
__global__ __launch_bounds__(kAuxBlock) void k_spatial(PassArgs A) {
  constexpr int kNb = 6;
  constexpr int CM = CT ? CT : kMaxC;
  __shared__ double red[kAuxBlock / 64];
  const ItemDev it = A.items[xcd_item(blockIdx.x, gridDim.x)];
  const GroupDev g = A.groups[it.group];
  const int tid = threadIdx.x;
  double lsum = 0.0;
  if ((g.priors & kPriorSpatial) && g.nbh > 0) {
    const int32_t* nbr = A.nbr + g.nbr_off;
    const int64_t V = g.V;
    const int C = CT ? CT : g.C;
    const float* fr = A.wsp + g.w_off + (int64_t)C * V;
    float* w_out = A.wsp + g.w_off;
    const float delta = A.model.huber_delta;
    for (int lv = tid; lv < it.nv; lv += blockDim.x) {
      const int v = it.v0 + lv;
      float mean[CM];
#pragma unroll
      for (int c = 0; c < CM; ++c) mean[c] = 0.0f;
      int cnt = 0;
      for (int q0 = 0; q0 < g.nbh; q0 += kNb) {
        int u[kNb];
#pragma unroll
        for (int j = 0; j < kNb; ++j) u[j] = q0 + j < g.nbh ? nbr[(int64_t)(q0 + j) * V + v] : -1;
        float t[kNb][CM];
#pragma unroll
        for (int j = 0; j < kNb; ++j) load_row<CT>(fr, u[j] >= 0 ? u[j] : v, C, t[j]);
#pragma unroll
        for (int j = 0; j < kNb; ++j) {
          const float on = u[j] >= 0 ? 1.0f : 0.0f;
          cnt += u[j] >= 0 ? 1 : 0;
#pragma unroll
          for (int c = 0; c < CM; ++c) mean[c] = fmaf(on, t[j][c], mean[c]);
        }
      }
      float own[CM];
      load_row<CT>(fr, v, C, own);
      float ls = 0.0f;
      const float icnt = cnt > 0 ? 1.0f / (float)cnt : 0.0f;
      float w[CM];
#pragma unroll
      for (int c = 0; c < CM; ++c) {
        w[c] = 0.0f;
        if (c < C && cnt > 0) {
          const float r = own[c] - mean[c] * icnt;
          const float ar = fabsf(r);
          ls += ar <= delta ? 0.5f * r * r : delta * (ar - 0.5f * delta);
          w[c] = (ar <= delta ? r : copysignf(delta, r)) * icnt;
        }
      }
      store_row<CT>(w_out, v, C, w);
      lsum += (double)ls;
    }
  }
  lsum = wave_sum_f64(lsum);
  if ((tid & 63) == 0) red[tid >> 6] = lsum;
  __syncthreads();
  if (tid == 0) {
    double s = 0.0;
    for (int i = 0; i < (int)(blockDim.x / 64); ++i) s += red[i];
    A.rec[g.rec_off + (int64_t)it.rec * g.rec_stride + kRecSpatial] = s;
  }
}

// ---------------------------------------------------------------------------
// whole-volume slabs: blend the per-slab constrained maps (Sec. 2.5)
// ---------------------------------------------------------------------------
// constrained quantities of voxel v: S0, fractions, unit directions, f_intra [, D]
template <int K, bool LD>
__device__ __forceinline__ void maps_at(const GroupDev& g, const float* th_all, int v, float (&m)[4 * K + 5 + (LD ? 2 : 0)]) {
  constexpr int C = K + 3;
  const float* th = th_all + g.micro_off;
  const int64_t V = g.V;
  m[0] = softplus_f(th[v]);
  float f[kMaxC];
  softmax_at(th, V, C, v, f);
#pragma unroll
  for (int c = 0; c < C; ++c) m[1 + c] = f[c];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const float x = th[(int64_t)row_v(C, k, 0) * V + v];
    const float y = th[(int64_t)row_v(C, k, 1) * V + v];
    const float z = th[(int64_t)row_v(C, k, 2) * V + v];
    const float n2 = fmaf(x, x, fmaf(y, y, z * z));
    const float in = n2 > 0.0f ? 1.0f / sqrtf(n2) : 0.0f;
    m[1 + C + 3 * k] = x * in;
    m[2 + C + 3 * k] = y * in;
    m[3 + C + 3 * k] = z * in;
  }
  m[1 + C + 3 * K] = sigmoid_f(th[(int64_t)row_fin(C, K) * V + v]);
  if (LD) {
    m[2 + C + 3 * K] = softplus_f(th[(int64_t)row_dpar(C, K) * V + v]);
    m[3 + C + 3 * K] = softplus_f(th[(int64_t)(row_dpar(C, K) + 1) * V + v]);
  }
}

// One thread per output voxel: one source is copied; two are blended with the
// heavier slab as reference (the lower slab on a tie), the other slab's fibres
// matched greedily by |cos| and sign-aligned.
template <int K, bool LD>
__global__ __launch_bounds__(256) void k_stitch(StitchArgs S) {
  constexpr int C = K + 3;
  constexpr int P = 4 * K + 5 + (LD ? 2 : 0);
  const int64_t o = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (o >= S.n_out) return;
  const int ga = S.src_g[o], gb = S.src_g[S.n_out + o];
  const float wa = S.src_w[o], wb = S.src_w[S.n_out + o];
  float ma[P];
  maps_at<K, LD>(S.groups[ga], S.th_micro, S.src_v[o], ma);
  float out[P];
  if (gb < 0) {
#pragma unroll
    for (int p = 0; p < P; ++p) out[p] = ma[p];
  } else {
    float mb[P];
    maps_at<K, LD>(S.groups[gb], S.th_micro, S.src_v[S.n_out + o], mb);
    const bool a_ref = wa >= wb;
    const float wr = a_ref ? wa : wb, wo = a_ref ? wb : wa;
    float r[P], q[P];
#pragma unroll
    for (int p = 0; p < P; ++p) {
      r[p] = a_ref ? ma[p] : mb[p];
      q[p] = a_ref ? mb[p] : ma[p];
      out[p] = wr * r[p] + wo * q[p];
    }
    int used = 0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const float rx = r[1 + C + 3 * k], ry = r[2 + C + 3 * k], rz = r[3 + C + 3 * k];
      float best = -1.0f, bdot = 0.0f, qf = 0.0f, qx = 0.0f, qy = 0.0f, qz = 0.0f;
      int bj = 0;
#pragma unroll
      for (int j = 0; j < K; ++j) {
        const float dot = rx * q[1 + C + 3 * j] + ry * q[2 + C + 3 * j] + rz * q[3 + C + 3 * j];
        if (!(used & (1 << j)) && fabsf(dot) > best) {
          best = fabsf(dot);
          bdot = dot;
          bj = j;
          qf = q[3 + j];
          qx = q[1 + C + 3 * j];
          qy = q[2 + C + 3 * j];
          qz = q[3 + C + 3 * j];
        }
      }
      used |= 1 << bj;
      const float sg = bdot < 0.0f ? -wo : wo;
      out[3 + k] = wr * r[3 + k] + wo * qf;
      const float dx = wr * rx + sg * qx, dy = wr * ry + sg * qy, dz = wr * rz + sg * qz;
      const float in = 1.0f / sqrtf(fmaf(dx, dx, fmaf(dy, dy, dz * dz)));
      out[1 + C + 3 * k] = dx * in;
      out[2 + C + 3 * k] = dy * in;
      out[3 + C + 3 * k] = dz * in;
    }
  }
#pragma unroll
  for (int p = 0; p < P; ++p) S.maps[(int64_t)p * S.n_out + o] = out[p];
}

// ---------------------------------------------------------------------------
// deterministic two-stage reduction of the item records
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_reduce1(ReduceArgs R) {
  __shared__ double part[4][64];
  const TileDev t = R.tiles[blockIdx.x];
  const GroupDev g = R.groups[t.group];
  const int f = threadIdx.x & 63, s = threadIdx.x >> 6;
  double acc = 0.0;
  if (f < t.nf) {
    // records r0 + s, r0 + s + 4, ...; eight loads in flight per step
    const double* base = R.rec + g.rec_off + t.f0 + f;
    const int64_t st = g.rec_stride;
    const int r1 = t.r0 + t.nr;
    int r = t.r0 + s;
    for (; r + 28 < r1; r += 32) {
      double a[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) a[i] = base[(int64_t)(r + 4 * i) * st];
      acc += ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
    }
    for (; r < r1; r += 4) acc += base[(int64_t)r * st];
  }
  part[s][f] = acc;
  __syncthreads();
  if (s == 0) R.part[(int64_t)t.out + f] = part[0][f] + part[1][f] + part[2][f] + part[3][f];
}

__global__ __launch_bounds__(256) void k_reduce2(ReduceArgs R) {
  __shared__ double part[4][64];
  __shared__ double calsq[3][4];
  const int gi = blockIdx.y, fc = blockIdx.x;
  const GroupDev g = R.groups[gi];
  const int nf_total = g.rec_stride;
  const int nfc = (nf_total + 63) / 64;
  if (fc >= nfc) return;
  const int f = threadIdx.x & 63, s = threadIdx.x >> 6;
  const int nrr = g.item_count > 0 ? (g.item_count + 63) / 64 : 0;
  double acc = 0.0;
  {
    // partial rows s, s + 4, ...; four loads in flight per step
    const double* pb = R.part + (int64_t)(g.tile_begin + fc * nrr) * 64 + f;
    int rr = s;
    for (; rr + 12 < nrr; rr += 16) {
      const double a0 = pb[(int64_t)rr * 64], a1 = pb[(int64_t)(rr + 4) * 64];
      const double a2 = pb[(int64_t)(rr + 8) * 64], a3 = pb[(int64_t)(rr + 12) * 64];
      acc += (a0 + a1) + (a2 + a3);
    }
    for (; rr < nrr; rr += 4) acc += pb[(int64_t)rr * 64];
  }
  part[s][f] = acc;
  const float* cal = R.th_cal + g.cal_off;
  float* gc = R.g_cal + g.cal_off;
  const int N = g.N, nb = g.n_bias;
  const bool cal_on = (g.priors & kPriorCal) != 0;
  // read before any thread of this block updates the calibration vector in place
  const float sigma_log = cal[nb + 2 * N];
  __shared__ float adam_sc[2];
  if (R.cal_adam && threadIdx.x == 0) adam_factors(R.step, R.lr, R.b1, R.b2, adam_sc[0], adam_sc[1], 1);
  // calibration L2 (Sec. 2.4) on block 0 of the group (precomputed when the
  // calibration vector is updated here)
  if (fc == 0 && !R.calsq) {
    double sa = 0.0, sb = 0.0, sw = 0.0;
    for (int i = threadIdx.x; i < nb; i += 256) sw += (double)cal[i] * cal[i];
    for (int i = threadIdx.x; i < N; i += 256) {
      sa += (double)cal[nb + i] * cal[nb + i];
      sb += (double)cal[nb + N + i] * cal[nb + N + i];
    }
    sa = wave_sum_f64(sa);
    sb = wave_sum_f64(sb);
    sw = wave_sum_f64(sw);
    if ((threadIdx.x & 63) == 0) {
      calsq[0][s] = sa;
      calsq[1][s] = sb;
      calsq[2][s] = sw;
    }
  }
  __syncthreads();
  if (s != 0) return;
  const int field = fc * 64 + f;
  if (field >= nf_total) return;
  const double tot = part[0][f] + part[1][f] + part[2][f] + part[3][f];
  const double M = g.V;
  const double sdata = g.mode == kMSE ? 2.0 * (double)g.invM : 1.0;
  float out = 0.0f;
  bool write = false;
  int dst = -1;
  if (field == kRecSigma) {
    dst = nb + 2 * N;
    out = g.mode == kNLL ? (float)(2.0 * N * M - tot) : 0.0f;
    write = true;
  } else if (field >= kRecBias && field < kRecBias + 10) {
    const int j = field - kRecBias;
    if (g.bias == 1) {
      dst = j;
      out = (float)(tot + (cal_on ? 2.0 * (double)R.model.lam_bias * cal[j] : 0.0));
      write = true;
    }
  } else if (field >= kRecAlpha && field < kRecAlpha + N) {
    const int n = field - kRecAlpha;
    dst = nb + n;
    out = (float)(sdata * tot + (cal_on ? 2.0 * (double)R.model.lam_alpha * cal[nb + n] : 0.0));
    write = true;
  } else if (field >= kRecAlpha + N && field < kRecAlpha + 2 * N) {
    const int n = field - kRecAlpha - N;
    dst = nb + N + n;
    out = (float)(sdata * tot + (cal_on ? 2.0 * (double)R.model.lam_beta * cal[nb + N + n] : 0.0));
    write = true;
  }
  if (write) {
    gc[dst] = out;
    if (!isfinite(out)) atomicOr(R.status, (uint32_t)kStNonfiniteGrad);
    if (R.cal_adam) {
      float p = R.th_cal_upd[g.cal_off + dst], m = R.m_cal[g.cal_off + dst], v = R.v_cal[g.cal_off + dst];
      adam_one(p, out, m, v, R.b1, R.b2, R.eps, adam_sc[0], adam_sc[1]);
      R.th_cal_upd[g.cal_off + dst] = p;
      R.m_cal[g.cal_off + dst] = m;
      R.v_cal[g.cal_off + dst] = v;
    }
  }
  if (fc == 0 && f == 0) {
    // loss terms from fields 0-7 of the LDS partials of this (first) field chunk
    auto part_sum = [&](int fld) { return part[0][fld] + part[1][fld] + part[2][fld] + part[3][fld]; };
    const double data = g.mode == kMSE
                            ? part_sum(kRecData) * (double)g.invM
                            : part_sum(kRecData) + 2.0 * (double)sigma_log * (double)N * M;
    const double sp = part_sum(kRecSpatial) * (double)R.model.lam_sp * g.invM;
    const double rp = part_sum(kRecRep) * (double)R.model.lam_rep * g.invM;
    const double sa = part_sum(kRecSparse) * (double)R.model.lam_sparse * g.invM;
    const double orp = part_sum(kRecOrphan) * (double)R.model.lam_orphan * g.invM;
    const double cnt = part_sum(kRecCont) * (double)R.model.lam_cont * g.invM;
    const double ord = part_sum(kRecOrder) * (double)R.model.lam_order * g.invM;
    const double tv = part_sum(kRecTV) * (double)R.model.lam_tv * g.invM;
    double cl = 0.0;
    if (cal_on) {
      const double* pre = R.calsq ? R.calsq + 3 * gi : nullptr;
      const double qa = pre ? pre[0] : calsq[0][0] + calsq[0][1] + calsq[0][2] + calsq[0][3];
      const double qb = pre ? pre[1] : calsq[1][0] + calsq[1][1] + calsq[1][2] + calsq[1][3];
      const double qw = pre ? pre[2] : calsq[2][0] + calsq[2][1] + calsq[2][2] + calsq[2][3];
      cl = (double)R.model.lam_alpha * qa + (double)R.model.lam_beta * qb +
           (double)R.model.lam_bias * qw;
    }
    double* L = R.loss + (int64_t)gi * kLossTerms;
    L[0] = data;
    L[1] = sp;
    L[2] = rp;
    L[3] = sa;
    L[4] = orp;
    L[5] = cnt;
    L[6] = ord;
    L[7] = cl;
    L[8] = tv;
    L[9] = data + sp + rp + sa + orp + cnt + ord + cl + tv;
    if (!isfinite(L[9])) atomicOr(R.status, (uint32_t)kStNonfiniteLoss);
    if (R.hist) {
      int slot = (R.hist_step[0] - R.hist_adv) % R.hist_len;
      if (slot < 0) slot += R.hist_len;
      double* H = R.hist + ((int64_t)slot * R.n_groups + gi) * kLossTerms;
#pragma unroll
      for (int i = 0; i < kLossTerms; ++i) H[i] = L[i];
    }
  }
}

// ---------------------------------------------------------------------------
// trilinear 8^3 log-bias gradient: dL/db(c) = sum_x w_c(x) dL/dlogB(x)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_bias_tri(ReduceArgs R, const int32_t* tri_groups) {
  __shared__ double red[4];
  const GroupDev g = R.groups[tri_groups[blockIdx.y]];
  const int cp = blockIdx.x;
  const int cidx[3] = {cp >> 6, (cp >> 3) & 7, cp & 7};
  const int nn[3] = {g.nx, g.ny, g.nz};
  int lo[3], hi[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (nn[a] == 1) {
      lo[a] = 0;
      hi[a] = cidx[a] == 0 ? 0 : -1;
    } else {
      const float sc = (float)(nn[a] - 1) / 7.0f;
      lo[a] = max(0, (int)ceilf((cidx[a] - 1) * sc));
      hi[a] = min(nn[a] - 1, (int)floorf((cidx[a] + 1) * sc));
    }
  }
  double acc = 0.0;
  const int ex = hi[0] - lo[0] + 1, ey = hi[1] - lo[1] + 1, ez = hi[2] - lo[2] + 1;
  if (ex > 0 && ey > 0 && ez > 0) {
    const int64_t tot = (int64_t)ex * ey * ez;
    const int32_t* grid = R.grid + g.grid_off;
    const float* glb = R.wsp + g.glb_off;
    for (int64_t q = threadIdx.x; q < tot; q += 256) {
      const int i = lo[0] + (int)(q / ((int64_t)ey * ez));
      const int j = lo[1] + (int)((q / ez) % ey);
      const int k = lo[2] + (int)(q % ez);
      const int v = grid[((int64_t)i * g.ny + j) * g.nz + k];
      if (v < 0) continue;
      const int ii[3] = {i, j, k};
      float w = 1.0f;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const float p = ii[a] * g.tri_sc[a];  // the coordinate of log_bias, bit for bit
        w *= fmaxf(0.0f, 1.0f - fabsf(p - (float)cidx[a]));
      }
      acc += (double)w * (double)glb[v];
    }
  }
  acc = wave_sum_f64(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double s = red[0] + red[1] + red[2] + red[3];
    const float* cal = R.th_cal + g.cal_off;
    const bool cal_on = (g.priors & kPriorCal) != 0;
    const float out = (float)(s + (cal_on ? 2.0 * (double)R.model.lam_bias * cal[cp] : 0.0));
    R.g_cal[g.cal_off + cp] = out;
    if (!isfinite(out)) atomicOr(R.status, (uint32_t)kStNonfiniteGrad);
    if (R.cal_adam) {
      float ss, ib;
      adam_factors(R.step, R.lr, R.b1, R.b2, ss, ib, 1);
      const int64_t i = g.cal_off + cp;
      float p = R.th_cal_upd[i], m = R.m_cal[i], v = R.v_cal[i];
      adam_one(p, out, m, v, R.b1, R.b2, R.eps, ss, ib);
      R.th_cal_upd[i] = p;
      R.m_cal[i] = m;
      R.v_cal[i] = v;
    }
  }
}

// ---------------------------------------------------------------------------
// optimisers
// ---------------------------------------------------------------------------
// Adam, PyTorch's form; t = step[0] + 1 is read by every block and the step
// counter is advanced afterwards by k_step_advance (stream order), so no
// block waits on another and no counter is contended.
// With advance != 0 the launch is a single block, which advances the step
// counter itself once every thread has used it.
__global__ __launch_bounds__(256) void k_adam(float* p, const float* g, float* m, float* v,
                                              int64_t n, float lr, float b1, float b2, float eps,
                                              int32_t* step, int vec4, int advance) {
  __shared__ float sc[2];
  if (threadIdx.x == 0) adam_factors(step, lr, b1, b2, sc[0], sc[1]);
  __syncthreads();
  const float step_size = sc[0], ibc2 = sc[1];
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t done = 0;
  if (vec4) {
    const int64_t n4 = n >> 2;
    float4* p4 = reinterpret_cast<float4*>(p);
    const float4* g4 = reinterpret_cast<const float4*>(g);
    float4* m4 = reinterpret_cast<float4*>(m);
    float4* v4 = reinterpret_cast<float4*>(v);
    for (int64_t i = tid; i < n4; i += stride) {
      float4 pp = p4[i], mm = m4[i], vv = v4[i];
      const float4 gg = g4[i];
      adam_one(pp.x, gg.x, mm.x, vv.x, b1, b2, eps, step_size, ibc2);
      adam_one(pp.y, gg.y, mm.y, vv.y, b1, b2, eps, step_size, ibc2);
      adam_one(pp.z, gg.z, mm.z, vv.z, b1, b2, eps, step_size, ibc2);
      adam_one(pp.w, gg.w, mm.w, vv.w, b1, b2, eps, step_size, ibc2);
      p4[i] = pp;
      m4[i] = mm;
      v4[i] = vv;
    }
    done = n4 << 2;
  }
  for (int64_t i = done + tid; i < n; i += stride) {
    float pp = p[i], mm = m[i], vv = v[i];
    adam_one(pp, g[i], mm, vv, b1, b2, eps, step_size, ibc2);
    p[i] = pp;
    m[i] = mm;
    v[i] = vv;
  }
  if (advance) {
    __syncthreads();
    if (threadIdx.x == 0) {
      step[0] = step[0] + 1;
      step[1] = 0;
    }
  }
}

__global__ void k_step_advance(int32_t* step) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    step[0] = step[0] + 1;
    step[1] = 0;
  }
}

__global__ __launch_bounds__(256) void k_rprop(float* p, const float* g, float* prev, float* st,
                                               int64_t n, float em, float ep, float smin,
                                               float smax) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    float gi = g[i];
    const float pr = gi * prev[i];
    float s = st[i];
    if (pr > 0.0f) s *= ep;
    else if (pr < 0.0f) s *= em;
    s = fminf(fmaxf(s, smin), smax);
    if (pr < 0.0f) gi = 0.0f;
    const float sg = gi > 0.0f ? 1.0f : (gi < 0.0f ? -1.0f : 0.0f);
    p[i] = p[i] - sg * s;
    prev[i] = gi;
    st[i] = s;
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_pass_maxn(const PassArgs& a, int K, int mode, int learn_d, int vpl, int maxN,
                            hipStream_t s) {
  switch (K) {
    case 1: return launch_pass_k<1>(a, mode, learn_d, vpl, maxN, s);
    case 2: return launch_pass_k<2>(a, mode, learn_d, vpl, maxN, s);
    case 3: return launch_pass_k<3>(a, mode, learn_d, vpl, maxN, s);
    case 4: return launch_pass_k<4>(a, mode, learn_d, vpl, maxN, s);
    case 5: return launch_pass_k<5>(a, mode, learn_d, vpl, maxN, s);
    case 6: return launch_pass_k<6>(a, mode, learn_d, vpl, maxN, s);
    default: return hipErrorInvalidValue;
  }
}

template <int CT>
static void launch_spatial_t(const PassArgs& a, dim3 grid, dim3 block, hipStream_t s) {
  const dim3 fgrid(grid.x + (a.calsq ? a.n_groups : 0));
  hipLaunchKernelGGL(k_fractions<CT>, fgrid, block, 0, s, a);
  hipLaunchKernelGGL(k_spatial<CT>, grid, block, 0, s, a);
}

hipError_t launch_spatial(const PassArgs& a, int n_items, int spatial_c, int max_nv, hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  // whole waves, one thread per voxel of the largest item, at most kAuxBlock;
  // k_spatial also writes each item's (zero) record when no group has the prior
  const dim3 grid(n_items), block(std::min(kAuxBlock, std::max(64, (max_nv + 63) / 64 * 64)));
  switch (spatial_c) {
    case 4: launch_spatial_t<4>(a, grid, block, s); break;
    case 5: launch_spatial_t<5>(a, grid, block, s); break;
    case 6: launch_spatial_t<6>(a, grid, block, s); break;
    case 7: launch_spatial_t<7>(a, grid, block, s); break;
    case 8: launch_spatial_t<8>(a, grid, block, s); break;
    case 9: launch_spatial_t<9>(a, grid, block, s); break;
    default: launch_spatial_t<0>(a, grid, block, s); break;
  }
  return hipGetLastError();
}

hipError_t launch_reduce(const ReduceArgs& a, int max_field_chunks, hipStream_t s) {
  if (a.n_tiles > 0) hipLaunchKernelGGL(k_reduce1, dim3(a.n_tiles), dim3(256), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (a.n_groups > 0 && max_field_chunks > 0)
    hipLaunchKernelGGL(k_reduce2, dim3(max_field_chunks, a.n_groups), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_bias_trilinear(const ReduceArgs& a, const int32_t* tri_groups, int n_tri,
                                 hipStream_t s) {
  if (n_tri <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_bias_tri, dim3(512, n_tri), dim3(256), 0, s, a, tri_groups);
  return hipGetLastError();
}

hipError_t launch_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1,
                       float b2, float eps, int32_t* step, hipStream_t s, bool advance) {
  const bool vec4 = ((reinterpret_cast<uintptr_t>(p) | reinterpret_cast<uintptr_t>(g) |
                      reinterpret_cast<uintptr_t>(m) | reinterpret_cast<uintptr_t>(v)) & 15) == 0;
  int64_t blocks = (n + 2047) / 2048;
  if (blocks < 1) blocks = 1;
  if (blocks > 4096) blocks = 4096;
  // a one-block update advances the counter itself (one launch instead of two)
  const int self_advance = advance && blocks == 1 ? 1 : 0;
  if (n > 0 || self_advance)
    hipLaunchKernelGGL(k_adam, dim3((unsigned)blocks), dim3(256), 0, s, p, g, m, v, n, lr, b1, b2,
                       eps, step, vec4 ? 1 : 0, self_advance);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !advance || self_advance) return e;
  hipLaunchKernelGGL(k_step_advance, dim3(1), dim3(64), 0, s, step);
  return hipGetLastError();
}

template <int K>
static hipError_t launch_stitch_k(const StitchArgs& a, int learn_d, hipStream_t s) {
  const unsigned blocks = (unsigned)((a.n_out + 255) / 256);
  if (learn_d)
    hipLaunchKernelGGL((k_stitch<K, true>), dim3(blocks), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL((k_stitch<K, false>), dim3(blocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_stitch(const StitchArgs& a, int K, int learn_d, hipStream_t s) {
  if (a.n_out <= 0) return hipSuccess;
  switch (K) {
    case 1: return launch_stitch_k<1>(a, learn_d, s);
    case 2: return launch_stitch_k<2>(a, learn_d, s);
    case 3: return launch_stitch_k<3>(a, learn_d, s);
    case 4: return launch_stitch_k<4>(a, learn_d, s);
    case 5: return launch_stitch_k<5>(a, learn_d, s);
    case 6: return launch_stitch_k<6>(a, learn_d, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_rprop(float* p, const float* g, float* prev, float* step, int64_t n, float em,
                        float ep, float smin, float smax, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 1023) / 1024;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_rprop, dim3((unsigned)blocks), dim3(256), 0, s, p, g, prev, step, n, em, ep,
                     smin, smax);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// the Eq. 9 special functions at given arguments, as the fused pass computes them
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_rician_terms(const float* z, float* li, float* omr, float* q,
                                                      int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    float o, qq;
    li[i] = log_i0e(z[i], o, qq);
    omr[i] = o;
    q[i] = qq;
  }
}

hipError_t launch_rician_terms(const float* z, float* li, float* omr, float* q, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_rician_terms, dim3((unsigned)blocks), dim3(256), 0, s, z, li, omr, q, n);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Static workspace of the allocation-free entry point (prism_loss_grad_noalloc)
// ---------------------------------------------------------------------------
// One array per device, held from the library's load until the process ends.
// In host code `scratch` names a host-side stand-in, not the device array:
// only the address hipGetSymbolAddress returns for the current device may be
// passed to kernels or copies.
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
hipError_t g_scratch_err[kMaxDevices] = {};
}  // namespace

hipError_t static_scratch_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return hipSuccess;
  int cur = -1;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return e;
  if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
  void* ptr = nullptr;
  e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e == hipSuccess && ptr == nullptr) e = hipErrorInvalidSymbol;
  if (e == hipSuccess) g_scratch_ptr[device] = ptr;
  g_scratch_err[device] = e;
  if (cur != device) (void)hipSetDevice(cur);
  return e;
}

void* static_scratch(int device, hipError_t* err) {
  if (device < 0 || device >= kMaxDevices) {
    *err = hipErrorInvalidDevice;
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  *err = g_scratch_ptr[device] ? hipSuccess
                               : (g_scratch_err[device] != hipSuccess ? g_scratch_err[device] : hipErrorNotInitialized);
  return g_scratch_ptr[device];
}

}  // namespace prism
