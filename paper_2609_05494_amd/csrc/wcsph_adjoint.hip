// wcsph_adjoint.hip -- reverse sweep of the WCSPH step (gradient of the
// summed wall-probe pressure impulse J = sum_k sum_n p_k^n dt_n with respect
// to alpha, delta and c0 at a fixed time-step table).
//
// One step is U* = E_A(U^n + dt/2 f(U^n)), U^{n+1} = E_B(U^n + dt f(U*)),
// f = rates (pair sums over fluid and Adami ghosts, ghosts from Shepard sums
// of the fluid), E = density band + wall / disk enforcement. Given the
// adjoint of U^{n+1} the sweep runs, per step and in reverse, two launches
// per evaluation:
//   k_adj_ghost (B)    transpose of E_B (adjoint of U^n, direct part, and the
//                      rate adjoints in the sorted slot order of U*), in the
//                      same launch as the ghost-state adjoints (pair terms
//                      seen by the fluid)
//   k_adj_fluid (B)    pull-form transpose of the rates at U* -> adjoint of U*
//   k_adj_ghost (A), k_adj_fluid (A) the same at U^n with the probe terms of
//                      step n
// Adjoints are FP32 per fluid particle (indexed by particle id); the
// coefficient gradients are reduced per block in FP64 in a fixed order.
// The sorted states, cell lists and pre-enforcement states of each
// evaluation come from the tape: written by the forward run itself when one
// segment covers it, else by a replay of each checkpoint segment.

#include "wcsph_adjoint.h"
#include "wcsph_launch.h"
#include "wcsph_kin.h"

namespace {

__device__ __forceinline__ float d_sqrt(float x) { return sqrtf(x); }
__device__ __forceinline__ float d_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float d_pow(float a, float b) { return powf(a, b); }

__device__ __forceinline__ PairK<float> pair_k(const InstParams& P) {
  PairK<float> k;
  k.h = P.h;
  k.inv_h = P.inv_h;
  k.four_h2 = P.four_h2;
  k.sigma = P.sigma;
  k.fgrad = P.fgrad;
  k.eta2h2 = P.eta2h2;
  k.alpha = P.alpha;
  k.delta = P.delta;
  k.two_h_c0 = P.two_h_c0;
  k.eps = P.eps_xsph;
  k.four_nu0 = P.four_nu0;
  return k;
}

__device__ __forceinline__ void cxy(const InstParams& P, uint32_t K, int& cx, int& cy) {
  const int local = (int)K - P.cell_off;
  cy = local / P.ncx;
  cx = local - cy * P.ncx;
}

__device__ __forceinline__ double block_sum(double v, double* sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += sh[w];
  __syncthreads();
  return t;
}

// Ghost density, P and c as functions of the ghost pressure (linear branch)
// and their derivatives.
struct GhostD {
  float rho, P, c, drho_dp, drho_dc0, dP_dp, dP_dc0, dc_drho, dc_dc0;
};
__device__ __forceinline__ GhostD ghost_d(const InstParams& P, float p) {
  GhostD g;
  const float c0 = P.c0;
  g.rho = P.rho0 * (1.0f + p * P.inv_rho0c02);
  g.drho_dp = 1.0f / (c0 * c0);
  g.drho_dc0 = -2.0f * p / (c0 * c0 * c0);
  const float r2 = g.rho * g.rho;
  g.P = p / r2;
  g.dP_dp = 1.0f / r2 - 2.0f * p / (r2 * g.rho) * g.drho_dp;
  g.dP_dc0 = -2.0f * p / (r2 * g.rho) * g.drho_dc0;
  g.c = c0 * powf(g.rho / P.rho0, P.c_exp);
  g.dc_drho = P.c_exp * g.c / g.rho;
  g.dc_dc0 = g.c / c0;
  return g;
}

}  // namespace

// Transpose of the update + enforcement of one evaluation for fluid particle
// i (by id). lam_out: adjoint of the evaluation's output state
// (x, y, vx, vy, rho); pre: pre-enforcement state taped by the forward
// kernel; te: time of the enforcement; hdt: dt/2 (eval A) or dt (eval B).
// (xd, vd): the disk at te (from the caller, the same for every particle).
// With WRITE, writes lam_base (+= when accumulate); returns the rate
// adjoints lf = hdt * (lam_pre_rho -> D, lam_pre_v -> a, lam_pre_r -> V).
template <bool WRITE>
__device__ __forceinline__ void adj_enforce_one(const InstParams& P, const AdjPtrs& a, int i, double xd, double vd,
                                                float hdt, int accumulate, float* lf) {
  const int n = P.nf;
  float lx = a.lam_out[i], ly = a.lam_out[n + i], lvx = a.lam_out[2 * n + i], lvy = a.lam_out[3 * n + i],
        lr = a.lam_out[4 * n + i];
  const double2 xp = a.pre_pos[i];
  const float4 vp = a.pre_vel[i];
  // density band
  if (vp.z < P.rho_lo || vp.z > P.rho_hi) lr = 0.0f;
  // walls (applied first in the forward)
  const double e = P.eps_wall;
  double xw = xp.x, yw = xp.y;
  float vxw = vp.x, vyw = vp.y;
  bool hx = false, hy = false;
  if (xw < e) { xw = e; vxw = -vxw; hx = true; }
  if (xw > P.L - e) { xw = P.L - e; vxw = -vxw; hx = true; }
  if (yw < e) { yw = e; vyw = -vyw; hy = true; }
  if (yw > P.W - e) { yw = P.W - e; vyw = -vyw; hy = true; }
  // disk: radial pull-out and reflection of the inward relative velocity
  if (P.nd > 0) {
    const double dx = xw - xd, dy = yw - P.disk_y0;
    const double d2 = dx * dx + dy * dy;
    if (d2 < P.R * P.R) {
      if (d2 > 0.0) {
        const double dd = sqrt(d2);
        const double nx = dx / dd, ny = dy / dd;
        const double s = (P.R + e) / dd;
        const double ux = (double)vxw - vd, uy = (double)vyw;
        const double w = ux * nx + uy * ny;
        // position: r = c + (R + eps) n  ->  d r / d r_w = s (I - n n^T)
        const double ln = lx * nx + ly * ny;
        double gx = s * (lx - ln * nx), gy = s * (ly - ln * ny);
        double gvx = lvx, gvy = lvy;
        if (w < 0.0) {
          // v = v_w - 2 w n: d v/d v_w = I - 2 n n^T;
          // d v/d r_w = -(2/|d|) [n (u^T P) + w P], P = I - n n^T
          const double lvn = lvx * nx + lvy * ny;
          gvx = lvx - 2.0 * lvn * nx;
          gvy = lvy - 2.0 * lvn * ny;
          const double un = ux * nx + uy * ny;
          const double pux = ux - un * nx, puy = uy - un * ny;   // P u
          const double plx = lvx - lvn * nx, ply = lvy - lvn * ny;  // P lam_v
          gx += -(2.0 / dd) * (pux * lvn + w * plx);
          gy += -(2.0 / dd) * (puy * lvn + w * ply);
        }
        lx = (float)gx;
        ly = (float)gy;
        lvx = (float)gvx;
        lvy = (float)gvy;
      } else {
        lx = 0.0f;
        ly = 0.0f;
      }
    }
  }
  if (hx) { lx = 0.0f; lvx = -lvx; }
  if (hy) { ly = 0.0f; lvy = -lvy; }
  if constexpr (WRITE) {
    float* lb = a.lam_base;
    if (accumulate) {
      // the five loads before any store (a store might otherwise alias the
      // next load, and each sum would wait for the one before it)
      const float b0 = lb[i], b1 = lb[n + i], b2 = lb[2 * n + i], b3 = lb[3 * n + i], b4 = lb[4 * n + i];
      lb[i] = b0 + lx; lb[n + i] = b1 + ly; lb[2 * n + i] = b2 + lvx; lb[3 * n + i] = b3 + lvy; lb[4 * n + i] = b4 + lr;
    } else {
      lb[i] = lx; lb[n + i] = ly; lb[2 * n + i] = lvx; lb[3 * n + i] = lvy; lb[4 * n + i] = lr;
    }
  }
  // rates: rho' = rho + h D, v' = v + h a, r' = r + h V
  lf[0] = hdt * lr;
  lf[1] = hdt * lvx;
  lf[2] = hdt * lvy;
  lf[3] = hdt * lx;
  lf[4] = hdt * ly;
}

// The enforcement transpose of fluid slot s, written straight into the
// sorted slot order of the taped evaluation (each fluid id holds one slot;
// ghost slots get zero): lam_base by id, the rate adjoints lam_s by slot.
__device__ __forceinline__ void adj_enforce_slot(const Dev& d, const InstParams& P, const AdjPtrs& a,
                                                 const TapeEval& te, int s,
                                                 double t_enf, float hdt, int accumulate) {
  if (s >= d.n_slots) return;
  double xd = 0.0, vd = 0.0, ad;
  if (P.nd > 0) kinematics(P, t_enf, xd, vd, ad);
  const int id = (int)te.id[s] - P.id0;
  float lf[5] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
  if (id >= 0 && id < P.nf) adj_enforce_one<true>(P, a, id, xd, vd, hdt, accumulate, lf);
  reinterpret_cast<float4*>(a.lam_s)[s] = make_float4(lf[0], lf[1], lf[2], lf[3]);
  a.lam_s[4 * d.n_slots + s] = lf[4];
}

// The 3x3 block of cells around (cx, cy) in a taped cell list as three row
// ranges; candidate c (rows bottom to top, cells left to right) maps to
// slot j and cell shift (dx, dy).
struct TRow {
  uint32_t rs, ms, me, re;
};
__device__ __forceinline__ TRow trow(const TapeEval& te, const InstParams& P, int cx, int cy, int dy) {
  TRow r = {0u, 0u, 0u, 0u};
  const int yy = cy + dy;
  if (yy < 0 || yy >= P.ncy) return r;
  const int xlo = max(cx - 1, 0), xhi = min(cx + 1, P.ncx - 1);
  const uint32_t k0 = (uint32_t)(P.cell_off + yy * P.ncx);
  r.rs = te.start[k0 + xlo];
  r.ms = te.start[k0 + cx];
  r.me = te.start[k0 + cx + 1];
  r.re = te.start[k0 + xhi + 1];
  return r;
}
// candidate counts below rows 1 and 2, and in all three rows
struct TCount {
  uint32_t n0, n01, n;
};
__device__ __forceinline__ TCount tcount(const TRow& r0, const TRow& r1, const TRow& r2) {
  TCount k;
  k.n0 = r0.re - r0.rs;
  k.n01 = k.n0 + (r1.re - r1.rs);
  k.n = k.n01 + (r2.re - r2.rs);
  return k;
}
// (three separate row variables: kept in registers, not indexed memory)
__device__ __forceinline__ void tcand(const TRow& r0, const TRow& r1, const TRow& r2, const TCount& k, uint32_t c,
                                      uint32_t& j, int& dx, int& dy) {
  const bool a0 = c < k.n0, a1 = c < k.n01;
  const TRow& r = a0 ? r0 : (a1 ? r1 : r2);
  j = r.rs + c - (a0 ? 0u : (a1 ? k.n0 : k.n01));
  dy = a0 ? -1 : (a1 ? 0 : 1);
  dx = j < r.ms ? -1 : (j < r.me ? 0 : 1);
}
#ifndef ADJ_FG
#define ADJ_FG 8  // lanes per fluid slot in the fluid adjoint kernel
#endif
#ifndef ADJ_LCAP
#define ADJ_LCAP 16  // entries of a lane's hit list in the fluid adjoint kernel
#endif

template <int G>
__device__ __forceinline__ float gsum(float v) {
  for (int o = 1; o < G; o <<= 1) v += __shfl_xor(v, o);
  return v;
}

// Ghost adjoints. For ghost g: the pair terms phi(i, g) of its fluid
// neighbours i give dL/d(rho_g, P_g, c_g, v_g); through the linear ghost
// density these become the adjoint of the ghost pressure (zero when the
// cavitation cutoff is active) and of c0. The ghost's Shepard sums are
// stored for the fluid pass. Extra threads compute the probes' Shepard sums.
#ifndef AG_L
#define AG_L 64  // lanes per ghost or probe (at most a wave: the sums are in-wave shuffles)
#endif
// One launch per evaluation carries both this pass (its first n_gb blocks)
// and the enforcement transpose of every slot (the blocks after them): the
// ghost items take their fluid neighbours' rate adjoints from the
// enforcement transpose recomputed per neighbour (a: the enforcement's
// adjoint pointers, t_enf, hdt), so neither waits for the other.
__global__ __launch_bounds__(256) void k_adj_ghost(Dev d, AdjPtrs a, TapeEval te, double t_eval, int n_gb,
                                                   double t_enf, float hdt, int acc_enf) {
  __shared__ double shd[4];
  // the instance's constants in LDS: read there in the candidate loop and
  // the enforcement transpose, where from global memory the compiler waited
  // for each field in turn
  __shared__ InstParams sP;
  {
    constexpr int NP = (int)(sizeof(InstParams) / 4);
    static_assert(sizeof(InstParams) % 4 == 0 && NP <= 256, "copy");
    if ((int)threadIdx.x < NP)
      reinterpret_cast<uint32_t*>(&sP)[threadIdx.x] = reinterpret_cast<const uint32_t*>(d.prm)[threadIdx.x];
    __syncthreads();
  }
  const InstParams& P = sP;
  if ((int)blockIdx.x >= n_gb) {
    adj_enforce_slot(d, P, a, te, ((int)blockIdx.x - n_gb) * 256 + (int)threadIdx.x, t_enf, hdt, acc_enf);
    return;
  }
  const int item = (int)((blockIdx.x * 256 + threadIdx.x) / AG_L);
  const int lane = (int)(threadIdx.x % AG_L);
  const int ng = P.nw + P.nd;
  double c0bar = 0.0;
  const PairK<float> k = pair_k(P);
  if (item < ng) {
    const int t = item;
    const uint32_t s = te.gslot[t];
    const uint32_t K = te.cell[s];
    const float4 pg = te.pv[s];
    const float4 ag = te.aux[s];  // rho_g, P_g, c_g, -m
    const bool disk = t >= P.nw;
    double xd, vd, ad;
    kinematics(P, t_eval, xd, vd, ad);
    const float awx = disk ? (float)ad : 0.0f;
    double xe = 0.0, ve = 0.0, ae_;  // the disk at the enforcement's time
    if (P.nd > 0) kinematics(P, t_enf, xe, ve, ae_);
    const float mg = -ag.w;
    int cx, cy;
    cxy(P, K, cx, cy);
    const TRow r0 = trow(te, P, cx, cy, -1), r1 = trow(te, P, cx, cy, 0), r2 = trow(te, P, cx, cy, 1);
    const TCount blk = tcount(r0, r1, r2);
    float gr = 0, gP = 0, gc = 0, gvx = 0, gvy = 0;
    float SW = 0, Sp = 0, Srx = 0, Sry = 0, Svx = 0, Svy = 0;
    for (uint32_t c = (uint32_t)lane; c < blk.n; c += AG_L) {
      uint32_t j;
      int dx, dy;
      tcand(r0, r1, r2, blk, c, j, dx, dy);
      float4 aj = te.aux[j];
      float4 pj = te.pv[j];
      uint32_t idr = te.id[j];
      // one round trip per candidate: the empty asm takes the loaded values,
      // so the compiler cannot defer the loads of pj and idr past the test
      asm("" : "+v"(aj.x), "+v"(aj.y), "+v"(aj.z), "+v"(aj.w), "+v"(pj.x), "+v"(pj.y), "+v"(pj.z), "+v"(pj.w),
          "+v"(idr));
      if (!(aj.w > 0.0f)) continue;
      // r_i - r_g for the pair phi(i, g)
      const float rx = (pj.x + (float)dx * P.dc) - pg.x, ry = (pj.y + (float)dy * P.dc) - pg.y;
      const float r2 = rx * rx + ry * ry;
      if (!(r2 < P.four_h2)) continue;
      PairIn<float> in;
      in.rx = rx; in.ry = ry; in.vx = pj.z - pg.z; in.vy = pj.w - pg.w;
      in.ra = aj.x; in.rb = ag.x; in.Pa = aj.y; in.Pb = ag.y; in.ca = aj.z; in.cb = ag.z;
      in.mb = mg; in.fl = 0.0f;
      PairGrad<float> g;
      // the neighbour's rate adjoints (its slot's lam_s entry)
      float lf[5];
      adj_enforce_one<false>(P, a, (int)idr - P.id0, xe, ve, hdt, 0, lf);
      pair_vjp(in, k, lf[0], lf[1], lf[2], lf[3], lf[4], g, d_sqrt, d_rcp);
      gr += g.rb;
      gP += g.P;
      gc += g.c;
      gvx -= g.vx;  // v = v_i - v_g
      gvy -= g.vy;
      // Shepard sums of the ghost (r_g - r_j = -(r_i - r_g))
      const float q = sqrtf(r2) * P.inv_h, sq = 1.0f - 0.5f * q, s2 = sq * sq;
      const float W = P.sigma * s2 * s2 * (2.0f * q + 1.0f);
      const float pj_ = aj.y * aj.x * aj.x;
      SW += W;
      Sp += pj_ * W;
      Srx += aj.x * (-rx) * W;
      Sry += aj.x * (-ry) * W;
      Svx += pj.z * W;
      Svy += pj.w * W;
    }
    gr = gsum<AG_L>(gr);
    gP = gsum<AG_L>(gP);
    gc = gsum<AG_L>(gc);
    gvx = gsum<AG_L>(gvx);
    gvy = gsum<AG_L>(gvy);
    SW = gsum<AG_L>(SW);
    Sp = gsum<AG_L>(Sp);
    Srx = gsum<AG_L>(Srx);
    Sry = gsum<AG_L>(Sry);
    Svx = gsum<AG_L>(Svx);
    Svy = gsum<AG_L>(Svy);
    if (lane == 0) {
      float pt = 0.0f, pbar = 0.0f, vax = 0.0f, vay = 0.0f;
      const float ax_ = 0.0f - awx, ay_ = P.gy;  // g - a_w
      if (SW > 0.0f) {
        pt = (Sp + ax_ * Srx + ay_ * Sry) / SW;
        vax = Svx / SW;
        vay = Svy / SW;
      }
      const float p = ag.y * ag.x * ag.x;  // taped ghost pressure
      const GhostD gd = ghost_d(P, p);
      const float pb = gr * gd.drho_dp + gP * gd.dP_dp + gc * gd.dc_drho * gd.drho_dp;
      c0bar += (double)(gr * gd.drho_dc0 + gP * gd.dP_dc0 + gc * (gd.dc_dc0 + gd.dc_drho * gd.drho_dc0));
      // v_g = 2 v_w - S_v / S_W; p_g = max(p~, p_cav)
      pbar = (SW > 0.0f && pt >= P.p_cav) ? pb : 0.0f;
      float* o = a.gadj + (size_t)s * 10;
      o[0] = pbar;
      o[1] = SW > 0.0f ? gvx : 0.0f;
      o[2] = SW > 0.0f ? gvy : 0.0f;
      o[3] = SW;
      o[4] = pt;
      o[5] = vax;
      o[6] = vay;
      o[7] = ax_;
      o[8] = ay_;
      o[9] = 0.0f;
    }
  } else if (item < ng + P.n_probes) {
    // probe Shepard sums at state n
    const int kk = item - ng;
    const uint32_t K = P.probe_cell[kk];
    int cx, cy;
    cxy(P, K, cx, cy);
    const TRow r0 = trow(te, P, cx, cy, -1), r1 = trow(te, P, cx, cy, 0), r2 = trow(te, P, cx, cy, 1);
    const TCount blk = tcount(r0, r1, r2);
    float SW = 0, Sp = 0;
    for (uint32_t c = (uint32_t)lane; c < blk.n; c += AG_L) {
      uint32_t j;
      int dx, dy;
      tcand(r0, r1, r2, blk, c, j, dx, dy);
      float4 aj = te.aux[j];
      float4 pj = te.pv[j];
      asm("" : "+v"(aj.x), "+v"(aj.y), "+v"(aj.z), "+v"(aj.w), "+v"(pj.x), "+v"(pj.y), "+v"(pj.z), "+v"(pj.w));
      if (!(aj.w > 0.0f)) continue;
      const float rx = P.probe_ox[kk] - (pj.x + (float)dx * P.dc), ry = P.probe_oy[kk] - (pj.y + (float)dy * P.dc);
      const float r2 = rx * rx + ry * ry;
      if (!(r2 < P.four_h2)) continue;
      const float q = sqrtf(r2) * P.inv_h, sq = 1.0f - 0.5f * q, s2 = sq * sq;
      const float W = P.sigma * s2 * s2 * (2.0f * q + 1.0f);
      SW += W;
      Sp += aj.y * aj.x * aj.x * W;
    }
    SW = gsum<AG_L>(SW);
    Sp = gsum<AG_L>(Sp);
    if (lane == 0) {
      a.padj[2 * kk] = SW;
      a.padj[2 * kk + 1] = SW > 0.0f ? Sp / SW : 0.0f;
    }
  }
  const double tot = block_sum(c0bar, shd);
  if (threadIdx.x == 0) a.theta_part[(size_t)blockIdx.x * 3 + 2] += tot;
}

// Fluid adjoints (pull form) for every fluid slot j of the taped
// evaluation: its own rates' dependence on its state, the dependence of its
// fluid neighbours' rates on its state, the ghost-mediated dependence
// through the Shepard sums, the XSPH identity and (probe_seed != 0) the
// probe terms; then the EOS chain. Output by particle id into lam_base
// (added, or set when accumulate == 0).
__global__ __launch_bounds__(256) void k_adj_fluid(Dev d, AdjPtrs a, TapeEval te, float probe_seed,
                                                    int accumulate, int block0) {
  // ADJ_FG lanes per slot (lane g of the group) share its 3x3 candidates
  __shared__ double shd[4];
  __shared__ uint32_t s_hits[ADJ_LCAP * 256];
  const InstParams& P = d.prm[0];
  const int s = (int)((blockIdx.x * 256 + threadIdx.x) / ADJ_FG);
  const int g = (int)(threadIdx.x % ADJ_FG);
  const int N = d.n_slots;
  const PairK<float> k = pair_k(P);
  double th_a = 0.0, th_d = 0.0, th_c = 0.0;
  if (s < N) {
    const float4 ai = te.aux[s];
    const int id = (int)te.id[s] - P.id0;
    if (ai.w > 0.0f && id >= 0 && id < P.nf) {
      const float4 pi = te.pv[s];
      const uint32_t K = te.cell[s];
      const float* ls = a.lam_s;
      const float4 l4 = reinterpret_cast<const float4*>(ls)[s];
      const float lD = l4.x, lax = l4.y, lay = l4.z, lVx = l4.w, lVy = ls[4 * N + s];
      const EosD<float> ei = eos_d<float>(ai.x, P.rho0, P.c0, P.gamma, P.p_cav, d_pow);
      // the XSPH identity term V = v + ... enters once (lane 0)
      float urx = 0, ury = 0, uvx = g == 0 ? lVx : 0.0f, uvy = g == 0 ? lVy : 0.0f, ur = 0, uP = 0, uc = 0,
            uc0 = 0;
      int cx, cy;
      cxy(P, K, cx, cy);
      const TRow r0 = trow(te, P, cx, cy, -1), r1 = trow(te, P, cx, cy, 0), r2 = trow(te, P, cx, cy, 1);
      const TCount blk = tcount(r0, r1, r2);
      // the in-support candidates go into a lane-private list in LDS (slot,
      // cell shift); the pair terms run over the list, so a wave runs them as
      // often as its longest list, not once per candidate position. Chunks of
      // ADJ_LCAP candidates per lane keep every list within its room; the
      // terms are summed in candidate order
      uint32_t* my = s_hits + threadIdx.x;
      const float4* ls4 = reinterpret_cast<const float4*>(ls);
      for (uint32_t c0 = (uint32_t)g; c0 < blk.n; c0 += ADJ_FG * ADJ_LCAP) {
        int cnt = 0;
        const uint32_t c1 = min(blk.n, c0 + ADJ_FG * ADJ_LCAP);
        // four candidates' positions in flight at once (past the chunk's
        // end a lane reads its first candidate again and records nothing)
        for (uint32_t cb = c0; cb < c1; cb += ADJ_FG * 4) {
          uint32_t jq[4];
          int dxq[4], dyq[4];
          float2 pq[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const uint32_t c = cb + ADJ_FG * (uint32_t)u;
            tcand(r0, r1, r2, blk, c < c1 ? c : c0, jq[u], dxq[u], dyq[u]);
            const float4 pc = te.pv[jq[u]];
            pq[u] = make_float2(pc.x, pc.y);
          }
          asm("" : "+v"(pq[0].x), "+v"(pq[0].y), "+v"(pq[1].x), "+v"(pq[1].y), "+v"(pq[2].x), "+v"(pq[2].y),
              "+v"(pq[3].x), "+v"(pq[3].y));
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            if (cb + ADJ_FG * (uint32_t)u >= c1) break;
            const float rxc = (pi.x - pq[u].x) - (float)dxq[u] * P.dc;
            const float ryc = (pi.y - pq[u].y) - (float)dyq[u] * P.dc;
            const bool hit = jq[u] != (uint32_t)s && rxc * rxc + ryc * ryc < P.four_h2;
            my[cnt * 256] = (jq[u] << 4) | ((uint32_t)(dyq[u] + 1) << 2) | (uint32_t)(dxq[u] + 1);
            cnt += hit ? 1 : 0;
          }
        }
        // the next hit's state is loaded while this one's terms are computed
        // (an empty list loads the lane's own slot, always in range)
        uint32_t cn = cnt > 0 ? my[0] : ((uint32_t)s << 4);
        float4 pn = te.pv[cn >> 4], an = te.aux[cn >> 4], ln = ls4[cn >> 4];
        float lyn = ls[4 * N + (cn >> 4)];
        for (int kk = 0; kk < cnt; ++kk) {
          const uint32_t code = cn;
          const uint32_t j = code >> 4;
          const int dx = (int)(code & 3u) - 1, dy = (int)((code >> 2) & 3u) - 1;
          const float4 pj = pn, aj = an, lj = ln;
          const float lyj = lyn;
          cn = my[min(kk + 1, cnt - 1) * 256];
          pn = te.pv[cn >> 4];
          an = te.aux[cn >> 4];
          ln = ls4[cn >> 4];
          lyn = ls[4 * N + (cn >> 4)];
          const float rx = (pi.x - pj.x) - (float)dx * P.dc;  // r_s - r_j
          const float ry = (pi.y - pj.y) - (float)dy * P.dc;
          const float r2 = rx * rx + ry * ry;
          const bool jfl = aj.w > 0.0f;
          // own rates: phi(s, j)
          PairIn<float> in;
          in.rx = rx; in.ry = ry; in.vx = pi.z - pj.z; in.vy = pi.w - pj.w;
          in.ra = ai.x; in.rb = aj.x; in.Pa = ai.y; in.Pb = aj.y; in.ca = ai.z; in.cb = aj.z;
          in.mb = fabsf(aj.w); in.fl = jfl ? 1.0f : 0.0f;
          PairGrad<float> gg;
          pair_vjp(in, k, lD, lax, lay, lVx, lVy, gg, d_sqrt, d_rcp);
          urx += gg.rx; ury += gg.ry; uvx += gg.vx; uvy += gg.vy; ur += gg.ra; uP += gg.P; uc += gg.c;
          th_a += (double)gg.alpha;
          th_d += (double)gg.delta;
          th_c += (double)gg.c0x;
          if (jfl) {
            // the neighbour's rates: phi(j, s), r = r_j - r_s
            PairIn<float> jn;
            jn.rx = -rx; jn.ry = -ry; jn.vx = pj.z - pi.z; jn.vy = pj.w - pi.w;
            jn.ra = aj.x; jn.rb = ai.x; jn.Pa = aj.y; jn.Pb = ai.y; jn.ca = aj.z; jn.cb = ai.z;
            jn.mb = ai.w; jn.fl = 1.0f;
            PairGrad<float> h;
            pair_vjp(jn, k, lj.x, lj.y, lj.z, lj.w, lyj, h, d_sqrt, d_rcp);
            urx -= h.rx; ury -= h.ry; uvx -= h.vx; uvy -= h.vy; ur += h.rb; uP += h.P; uc += h.c;
          } else {
            // ghost j: this particle enters the ghost's Shepard sums
            const float* gq = a.gadj + (size_t)j * 10;
            const float SW = gq[3];
            if (SW > 0.0f) {
              const float pbar = gq[0], vbx = gq[1], vby = gq[2], pt = gq[4], vax = gq[5], vay = gq[6];
              const float gx = gq[7], gy = gq[8];
              const float ddx = -rx, ddy = -ry;  // d = r_g - r_s
              const float q = sqrtf(r2) * P.inv_h, sq = 1.0f - 0.5f * q, s2 = sq * sq;
              const float W = P.sigma * s2 * s2 * (2.0f * q + 1.0f);
              const float F = -P.fgrad * s2 * sq;
              const float ad_ = gx * ddx + gy * ddy;
              const float iw = 1.0f / SW;
              ur += pbar * (ei.dp + ad_) * W * iw;
              const float cf = -(ei.p + ai.x * ad_ - pt) * F * iw;
              const float vv = vbx * (pi.z - vax) + vby * (pi.w - vay);
              urx += pbar * (cf * ddx - ai.x * W * iw * gx) + vv * F * ddx * iw;
              ury += pbar * (cf * ddy - ai.x * W * iw * gy) + vv * F * ddy * iw;
              uvx -= vbx * W * iw;
              uvy -= vby * W * iw;
              uc0 += pbar * ei.dpdc0 * W * iw;
            }
          }
        }
      }
      if (probe_seed != 0.0f && g == 0) {
        for (int kk = 0; kk < P.n_probes; ++kk) {
          const float SW = a.padj[2 * kk];
          if (!(SW > 0.0f)) continue;
          int px, py;
          cxy(P, P.probe_cell[kk], px, py);
          if (abs(px - cx) > 1 || abs(py - cy) > 1) continue;
          const float ddx = (P.probe_ox[kk] + (float)(px - cx) * P.dc) - pi.x;  // d = r_k - r_s
          const float ddy = (P.probe_oy[kk] + (float)(py - cy) * P.dc) - pi.y;
          const float r2 = ddx * ddx + ddy * ddy;
          if (!(r2 < P.four_h2)) continue;
          const float q = sqrtf(r2) * P.inv_h, sq = 1.0f - 0.5f * q, s2 = sq * sq;
          const float W = P.sigma * s2 * s2 * (2.0f * q + 1.0f);
          const float F = -P.fgrad * s2 * sq;
          const float iw = probe_seed / SW;
          ur += ei.dp * W * iw;
          urx += -(ei.p - a.padj[2 * kk + 1]) * F * ddx * iw;
          ury += -(ei.p - a.padj[2 * kk + 1]) * F * ddy * iw;
          uc0 += ei.dpdc0 * W * iw;
        }
      }
      // fixed-order quad sums
      urx = gsum<ADJ_FG>(urx);
      ury = gsum<ADJ_FG>(ury);
      uvx = gsum<ADJ_FG>(uvx);
      uvy = gsum<ADJ_FG>(uvy);
      ur = gsum<ADJ_FG>(ur);
      uP = gsum<ADJ_FG>(uP);
      uc = gsum<ADJ_FG>(uc);
      uc0 = gsum<ADJ_FG>(uc0);
      if (g == 0) {
        // EOS chain: P(rho; c0), c(rho; c0)
        ur += uP * ei.dPdr + uc * ei.dcdr;
        uc0 += uP * ei.dPdc0 + uc * ei.dcdc0;
        th_c += (double)uc0;
        const int n = P.nf;
        float* lb = a.lam_base;
        if (accumulate) {
          // the five loads before any store (as in the enforcement transpose)
          const float b0 = lb[id], b1 = lb[n + id], b2 = lb[2 * n + id], b3 = lb[3 * n + id], b4 = lb[4 * n + id];
          lb[id] = b0 + urx; lb[n + id] = b1 + ury; lb[2 * n + id] = b2 + uvx; lb[3 * n + id] = b3 + uvy;
          lb[4 * n + id] = b4 + ur;
        } else {
          lb[id] = urx; lb[n + id] = ury; lb[2 * n + id] = uvx; lb[3 * n + id] = uvy; lb[4 * n + id] = ur;
        }
      }
    }
  }
  const double ta = block_sum(th_a, shd), td = block_sum(th_d, shd), tc = block_sum(th_c, shd);
  if (threadIdx.x == 0) {
    double* o = a.theta_part + (size_t)(block0 + blockIdx.x) * 3;
    o[0] += ta;
    o[1] += td;
    o[2] += tc;
  }
}

// theta += sum of the per-block running sums (FP64, fixed order: lane l
// adds blocks l, l + 64, ... in order, then a butterfly over the wave); once,
// after the reverse sweep.
__global__ void k_adj_theta(AdjPtrs a, int nblk) {
  if (blockIdx.x != 0) return;
  double t[3];
  for (int k = 0; k < 3; ++k) {
    double v = 0.0;
    for (int b = (int)threadIdx.x; b < nblk; b += 64) v += a.theta_part[3 * b + k];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    t[k] = v;
  }
  if (threadIdx.x == 0) {
    a.theta[0] += t[0];
    a.theta[1] += t[1];
    a.theta[2] += t[2];
  }
}

// ---------------------------------------------------------------------------
// Backward pass of one evaluation's rates (ghost adjoints, fluid adjoints,
// coefficient partials added to each block's running sums). lam_s (by
// slot) -> lam_base (by id).
static int adj_ghost_blocks(int n_ghost_probe) { return (n_ghost_probe * AG_L + 255) / 256; }
static int adj_fluid_blocks(int n_slots) { return (n_slots * ADJ_FG + 255) / 256; }

int wc_adj_partial_blocks(int n_ghost_probe, int n_slots) {
  return adj_ghost_blocks(n_ghost_probe) + adj_fluid_blocks(n_slots);
}

void wc_enqueue_adj_eval(const Dev& d, const AdjPtrs& ae, const AdjPtrs& ar, const TapeEval& te, double t_enf,
                         float hdt, bool acc_enf, double t_eval, float probe_seed, bool acc_rates, hipStream_t st) {
  const int ngb = adj_ghost_blocks(ae.n_ghost_probe);
  const int neb = (d.n_slots + 255) / 256;
  k_adj_ghost<<<ngb + neb, 256, 0, st>>>(d, ae, te, t_eval, ngb, t_enf, hdt, acc_enf ? 1 : 0);
  const int nfb = adj_fluid_blocks(d.n_slots);
  k_adj_fluid<<<nfb, 256, 0, st>>>(d, ar, te, probe_seed, acc_rates ? 1 : 0, ngb);
}

void wc_enqueue_adj_theta(const AdjPtrs& a, int nblk, hipStream_t st) { k_adj_theta<<<1, 64, 0, st>>>(a, nblk); }

