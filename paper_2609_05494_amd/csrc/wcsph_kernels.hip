// wcsph_kernels.hip -- HIP kernels of the planar WCSPH step for gfx950.
//
// One step = two evaluations (predictor-corrector). Each evaluation runs:
//   k_kin      clock, prescribed disk kinematics, disk-ring placement and
//              the ring's bucket slots for the next sort
//   k_scan     exclusive scan of the per-cell counts -> cell ranges
//   k_scatter  every slot into its cell bucket
//   k_permute  stable rank inside the bucket (by old slot) and gather of the
//              state into sorted order; per-particle EOS (P = p/rho^2, c)
//   k_ghost    Adami-Shepard ghost state on walls and ring, probes (eval A),
//              v_max of the ghosts (eval A), work of the ring (eval B)
//   k_pair     pair sums over the 3x3 cells (continuity + delta, pressure +
//              AV + laminar, XSPH) fused with the predictor / corrector,
//              density band, enforcement, new cell key and bucket slot
// Pair arithmetic is FP32 on cell-relative offsets; time, kinematics,
// enforcement geometry and diagnostics are FP64.

#include "wcsph_launch.h"

namespace {

template <bool BATCH>
__device__ __forceinline__ int inst_at(const Buf& b, int s) {
  if constexpr (BATCH) return (int)b.inst[s];
  else return 0;
}

// Spread consecutive blocks over the 8 XCDs in contiguous chunks: hardware
// dispatches block b to XCD b % 8, so logical chunk x (one L2) is served by
// the blocks with b % 8 == x.
__device__ __forceinline__ int xcd_block(int bid, int nblk) {
  const int q = nblk >> 3, r = nblk & 7, x = bid & 7;
  return x * q + min(x, r) + (bid >> 3);
}

__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float fast_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }

// Prescribed disk motion along +x (velocity ramp, then constant deceleration
// or quadratic drag), FP64 closed forms.
__device__ void kinematics(const InstParams& P, double t, double& x, double& v, double& a) {
  const double v0 = P.kin_v0, tr = P.kin_t_ramp;
  if (t < tr) {
    v = v0 * t / tr;
    a = v0 / tr;
    x = P.disk_x0 + 0.5 * v0 * t * t / tr;
    return;
  }
  const double tau = t - tr, xr = P.disk_x0 + 0.5 * v0 * tr;
  if (P.kin_mode == 1) {
    const double k = P.kin_coef;
    v = v0 / (1.0 + k * v0 * tau);
    a = -k * v * v;
    x = k > 0.0 ? xr + log1p(k * v0 * tau) / k : xr + v0 * tau;
    return;
  }
  const double ad = P.kin_coef;
  if (ad > 0.0 && tau >= v0 / ad) {
    v = 0.0;
    a = 0.0;
    x = xr + 0.5 * v0 * v0 / ad;
    return;
  }
  v = v0 - ad * tau;
  a = -ad;
  x = xr + v0 * tau - 0.5 * ad * tau * tau;
}

// Tait pressure with the cavitation cutoff, P = p / rho^2 and the sound speed
// c0 (rho/rho0)^((gamma-1)/2); written through log1p/expm1 so that p stays
// accurate near rho0 in FP32.
__device__ __forceinline__ void fluid_eos(const InstParams& P, float rho, float& Pq, float& c) {
  const float l = log1pf((rho - P.rho0) / P.rho0);
  const float p = fmaxf(P.B * expm1f(P.gamma * l), P.p_cav);
  Pq = p / (rho * rho);
  c = P.c0 * expf(P.c_exp * l);
}

// Wendland C2 (2D): W = sigma (1-q/2)^4 (2q+1); grad_i W = F r_ij,
// F = -fgrad (1-q/2)^3.
__device__ __forceinline__ void wendland(const InstParams& P, float r2, float& W, float& F) {
  const float q = fast_sqrt(r2) * P.inv_h;
  const float s = 1.0f - 0.5f * q;
  const float s2 = s * s;
  W = P.sigma * s2 * s2 * (2.0f * q + 1.0f);
  F = -P.fgrad * s2 * s;
}

__device__ __forceinline__ void cell_xy(const InstParams& P, uint32_t K, int& cx, int& cy) {
  const int local = (int)K - P.cell_off;
  cy = local / P.ncx;
  cx = local - cy * P.ncx;
}

// Encode an FP64 position into (cell, FP32 offset inside the cell).
__device__ __forceinline__ void encode_axis(double x, double lo, double dcd, float dc, int n, int& c,
                                            float& o) {
  const double u = x - lo;
  c = (int)floor(u / dcd);
  if (c < 0) c = 0;
  if (c > n - 1) c = n - 1;
  o = (float)(u - (double)c * dcd);
  if (o >= dc && c < n - 1) {
    o -= dc;
    c += 1;
  }
}

// Keep an offset inside [0, dc) after a move, shifting the cell index.
__device__ __forceinline__ void renorm(float& o, int& c, float dc) {
  if (o < 0.0f) {
    o += dc;
    c -= 1;
    if (o >= dc) {  // a tiny negative offset rounded up to dc
      o -= dc;
      c += 1;
    }
  } else if (o >= dc) {
    o -= dc;
    c += 1;
  }
  if (o < 0.0f || o >= dc) {  // a jump of more than one cell
    const float n = floorf(o / dc);
    c += (int)n;
    o -= n * dc;
    if (o < 0.0f) o = 0.0f;
    if (o >= dc) o = 0.0f;
  }
}

__device__ __forceinline__ double step_dt(const Dev& d, const InstParams& P, const Clock& C) {
  if (d.n_dt > 0) {
    const long long k = C.step - d.dt_step0;
    if (k >= 0 && k < d.n_dt) return d.dt_table[k];
  }
  const float vm = __uint_as_float(C.vmax_bits);
  return P.cfl * P.hd / (P.c0d + (double)vm);
}

__device__ __forceinline__ float wave_max(float v) {
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
  return v;
}
__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// Max of |v| into the instance accumulator: one atomic per wave when the
// wave holds a single instance, else one per lane.
template <bool BATCH>
__device__ __forceinline__ void vmax_update(Clock* clk, int inst, bool act, float v) {
  const float m = act ? v : 0.0f;
  if constexpr (BATCH) {
    const int i0 = __shfl(inst, 0);
    if (__all(inst == i0)) {
      const float w = wave_max(m);
      if ((threadIdx.x & 63) == 0 && w > 0.0f) atomicMax(&clk[i0].vmax_bits, __float_as_uint(w));
    } else if (act && m > 0.0f) {
      atomicMax(&clk[inst].vmax_bits, __float_as_uint(m));
    }
  } else {
    const float w = wave_max(m);
    if ((threadIdx.x & 63) == 0 && w > 0.0f) atomicMax(&clk[0].vmax_bits, __float_as_uint(w));
  }
}

template <bool BATCH>
__device__ __forceinline__ void count_hits(Clock* clk, int inst, bool clamp, bool enf) {
  if constexpr (BATCH) {
    if (clamp) atomicAdd(&clk[inst].n_clamp, 1ull);
    if (enf) atomicAdd(&clk[inst].n_enforce, 1ull);
  } else {
    const unsigned long long bc = __ballot(clamp), be = __ballot(enf);
    if ((threadIdx.x & 63) == 0) {
      if (bc) atomicAdd(&clk[0].n_clamp, (unsigned long long)__popcll(bc));
      if (be) atomicAdd(&clk[0].n_enforce, (unsigned long long)__popcll(be));
    }
  }
}

struct PairAcc {
  float D, ax, ay, Vx, Vy;
};

// Sum the pair law of fluid slot s over its 3x3 block of cells
// (rows bottom to top, cells left to right, sorted order inside a cell).
__device__ __forceinline__ void pair_sums(const Dev& d, const InstParams& P, const Buf& sb, int s,
                                          uint32_t K, float4 pi, float4 ai, PairAcc& acc) {
  const float rhoi = ai.x, Pi = ai.y, ci = ai.z;
  int cx, cy;
  cell_xy(P, K, cx, cy);
  for (int dy = -1; dy <= 1; ++dy) {
    const int yy = cy + dy;
    if (yy < 0 || yy >= P.ncy) continue;
    const float shy = (float)dy * P.dc;
    for (int dx = -1; dx <= 1; ++dx) {
      const int xx = cx + dx;
      if (xx < 0 || xx >= P.ncx) continue;
      const float shx = (float)dx * P.dc;
      const uint32_t K2 = (uint32_t)(P.cell_off + yy * P.ncx + xx);
      const uint32_t j0 = d.start[K2], j1 = d.start[K2 + 1];
      for (uint32_t j = j0; j < j1; ++j) {
        const float4 pj = sb.pv[j];
        const float rx = (pi.x - pj.x) - shx;  // r_i - r_j
        const float ry = (pi.y - pj.y) - shy;
        const float r2 = rx * rx + ry * ry;
        if (!(r2 < P.four_h2) || j == (uint32_t)s) continue;
        const float4 aj = sb.aux[j];
        float W, F;
        wendland(P, r2, W, F);
        const float vxij = pi.z - pj.z, vyij = pi.w - pj.w;
        const float vr = vxij * rx + vyij * ry;
        const bool fl = aj.w > 0.0f;
        const float mj = fabsf(aj.w);
        const float rsum = rhoi + aj.x;       // 2 rho_bar
        const float den = r2 + P.eta2h2;      // r^2 + eta^2 h^2
        const float inv = fast_rcp(den * rsum);
        // Monaghan AV: -alpha c_bar mu / rho_bar = -alpha (c_i + c_j) h vr inv
        const float piav = vr < 0.0f ? -P.alpha * (ci + aj.z) * P.h * vr * inv : 0.0f;
        const float mF = mj * F;
        acc.D += mF * vr;
        const float sp = Pi + aj.y + piav;
        acc.ax -= mF * sp * rx;
        acc.ay -= mF * sp * ry;
        // laminar (Lo-Shao): 4 nu0 m_j F r^2 / ((rho_i + rho_j)(r^2 + eta^2 h^2)) v_ij
        const float lam = P.four_nu0 * mF * r2 * inv;
        acc.ax += lam * vxij;
        acc.ay += lam * vyij;
        if (fl) {
          // delta diffusion 2 delta h c0 (m_j / rho_j)(rho_i - rho_j) F
          acc.D += P.two_delta_h_c0 * mj * fast_rcp(aj.x) * (rhoi - aj.x) * F;
          // XSPH eps (m_j / rho_bar) W (v_j - v_i); 1 / rho_bar = 2 den inv
          const float w = P.eps_xsph * mj * 2.0f * den * inv * W;
          acc.Vx -= w * vxij;
          acc.Vy -= w * vyij;
        }
      }
    }
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// Clock, kinematics and disk-ring placement; one block per instance.
template <int MODE>
__global__ __launch_bounds__(256) void k_kin(Dev d, Buf pre) {
  const int i = blockIdx.x;
  const InstParams& P = d.prm[i];
  Clock& C = d.clk[i];
  __shared__ double sh[3];
  if (threadIdx.x == 0) {
    double te;
    if (MODE == EV_A) {
      C.t = C.t_next;
      C.step += 1;
      te = C.t;
    } else if (MODE == EV_B) {
      const double dt = step_dt(d, P, C);
      C.dt = dt;
      C.vmax_used = (double)__uint_as_float(C.vmax_bits);
      C.vmax_bits = 0u;
      const long long row = (long long)i * WC_HIST_CAP + (C.step % WC_HIST_CAP);
      d.hist_t[row] = C.t;
      d.hist_dt[row] = dt;
      te = C.t + 0.5 * dt;
    } else {
      te = C.t_next;
    }
    double x, v, a;
    kinematics(P, te, x, v, a);
    C.t_eval = te;
    C.xd = x;
    C.vd = v;
    C.ad = a;
    sh[0] = x;
  }
  __syncthreads();
  const double xc = sh[0];
  for (int k = threadIdx.x; k < P.nd; k += blockDim.x) {
    double sn, cs;
    sincos(2.0 * M_PI * (double)k / (double)P.nd, &sn, &cs);
    const double x = xc + P.R * cs, y = P.disk_y0 + P.R * sn;
    int cx, cy;
    float ox, oy;
    encode_axis(x, P.x_lo, P.dcd, P.dc, P.ncx, cx, ox);
    encode_axis(y, P.y_lo, P.dcd, P.dc, P.ncy, cy, oy);
    const uint32_t key = (uint32_t)(P.cell_off + cy * P.ncx + cx);
    const uint32_t s = d.gslot[P.gmap0 + P.nw + k];
    pre.cell[s] = key;
    pre.pv[s] = make_float4(ox, oy, 0.0f, 0.0f);
    pre.bslot[s] = atomicAdd(&d.count[key], 1u);
  }
}

// Exclusive scan of count -> start over all cells; count is re-armed with the
// static wall-ghost occupancy for the next sort. One block.
__global__ __launch_bounds__(1024) void k_scan(Dev d) {
  __shared__ uint32_t wsum[16];
  const int n = d.n_cells;
  const int t = threadIdx.x;
  const int chunk = (n + 1023) / 1024;
  const int lo = min(n, t * chunk), hi = min(n, lo + chunk);
  uint32_t s = 0;
  for (int c = lo; c < hi; ++c) s += d.count[c];
  // inclusive scan of per-thread sums: wave level then across waves
  uint32_t incl = s;
  const int lane = t & 63, wv = t >> 6;
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t u = __shfl_up(incl, o);
    if (lane >= o) incl += u;
  }
  if (lane == 63) wsum[wv] = incl;
  __syncthreads();
  uint32_t base = 0;
  for (int w = 0; w < wv; ++w) base += wsum[w];
  uint32_t run = base + incl - s;
  for (int c = lo; c < hi; ++c) {
    const uint32_t v = d.count[c];
    d.start[c] = run;
    run += v;
    d.count[c] = d.wallcount[c];
  }
  if (t == 1023) d.start[n] = base + incl;
}

// Every slot into its bucket: tmp[start[key] + bucket slot] = slot.
template <bool BATCH>
__global__ __launch_bounds__(WC_BLOCK) void k_scatter(Dev d, Buf pre) {
  const int s = blockIdx.x * WC_BLOCK + threadIdx.x;
  if (s >= d.n_slots) return;
  const InstParams& P = d.prm[inst_at<BATCH>(pre, s)];
  const uint32_t K = pre.cell[s];
  const int local = (int)pre.id[s] - P.id0;
  uint32_t b;
  if (local >= P.nf && local < P.nf + P.nw) b = d.wrank[P.gmap0 + local - P.nf];
  else b = pre.bslot[s];
  const uint32_t dst = d.start[K] + b;
  if (dst < d.start[K + 1] && dst < (uint32_t)d.n_slots) d.tmp[dst] = (uint32_t)s;
  else atomicOr(&d.clk[0].bad, 2u);
}

// Stable rank inside the bucket and gather into sorted order. In eval B the
// state at time n (pre2, same slot order as pre) is permuted alongside.
template <int MODE, bool BATCH>
__global__ __launch_bounds__(WC_BLOCK) void k_permute(Dev d, Buf pre, Buf out, Buf pre2, Buf out2) {
  const int p = blockIdx.x * WC_BLOCK + threadIdx.x;
  if (p >= d.n_slots) return;
  const uint32_t e = d.tmp[p];
  if (e >= (uint32_t)d.n_slots) {
    atomicOr(&d.clk[0].bad, 4u);
    return;
  }
  const uint32_t K = pre.cell[e];
  const uint32_t lo = d.start[K], hi = min(d.start[K + 1], (uint32_t)d.n_slots);
  uint32_t rank = 0;
  for (uint32_t t = lo; t < hi; ++t) rank += d.tmp[t] < e ? 1u : 0u;
  const uint32_t dst = lo + rank;
  const int inst = inst_at<BATCH>(pre, e);
  const InstParams& P = d.prm[inst];
  const uint32_t id = pre.id[e];
  const float4 pv = pre.pv[e];
  const float rho = pre.aux[e].x;
  const int local = (int)id - P.id0;
  float4 a;
  if (local < P.nf) {
    float Pq, c;
    fluid_eos(P, rho, Pq, c);
    a = make_float4(rho, Pq, c, P.m_fluid);
  } else {
    const int g = local - P.nf;
    a = make_float4(rho, 0.0f, 0.0f, g < P.nw ? -P.m_wall : -P.m_disk);
    d.gslot[P.gmap0 + g] = dst;
  }
  out.cell[dst] = K;
  out.id[dst] = id;
  out.pv[dst] = pv;
  out.aux[dst] = a;
  if constexpr (BATCH) out.inst[dst] = (uint16_t)inst;
  d.perm[dst] = e;
  if (MODE == EV_B) {
    out2.cell[dst] = pre2.cell[e];
    out2.id[dst] = pre2.id[e];
    out2.pv[dst] = pre2.pv[e];
    out2.aux[dst] = pre2.aux[e];
    if constexpr (BATCH) out2.inst[dst] = (uint16_t)inst;
  }
}

// Shepard sums over the fluid around an encoded point (cell K, offset o).
struct Shep {
  float W, p, rx, ry, vx, vy;
};
__device__ __forceinline__ Shep shepard(const Dev& d, const InstParams& P, const Buf& sb, uint32_t K,
                                        float ox, float oy) {
  Shep S = {0, 0, 0, 0, 0, 0};
  int cx, cy;
  cell_xy(P, K, cx, cy);
  for (int dy = -1; dy <= 1; ++dy) {
    const int yy = cy + dy;
    if (yy < 0 || yy >= P.ncy) continue;
    const float shy = (float)dy * P.dc;
    for (int dx = -1; dx <= 1; ++dx) {
      const int xx = cx + dx;
      if (xx < 0 || xx >= P.ncx) continue;
      const float shx = (float)dx * P.dc;
      const uint32_t K2 = (uint32_t)(P.cell_off + yy * P.ncx + xx);
      const uint32_t j0 = d.start[K2], j1 = d.start[K2 + 1];
      for (uint32_t j = j0; j < j1; ++j) {
        const float4 aj = sb.aux[j];
        if (!(aj.w > 0.0f)) continue;  // fluid only
        const float4 pj = sb.pv[j];
        const float rx = (ox - pj.x) - shx;  // r_g - r_j
        const float ry = (oy - pj.y) - shy;
        const float r2 = rx * rx + ry * ry;
        if (!(r2 < P.four_h2)) continue;
        float W, F;
        wendland(P, r2, W, F);
        const float pj_ = aj.y * aj.x * aj.x;  // p = P rho^2
        S.W += W;
        S.p += pj_ * W;
        S.rx += aj.x * rx * W;
        S.ry += aj.x * ry * W;
        S.vx += pj.z * W;
        S.vy += pj.w * W;
      }
    }
  }
  return S;
}

// Adami ghost state (walls and ring), probes, ghost v_max and ring work.
// Block table entry: (instance, first ghost, ghost count, kind); kind 1 is
// the instance's ring + probe block.
template <int MODE, bool BATCH>
__global__ __launch_bounds__(WC_GHOST_BLOCK) void k_ghost(Dev d, Buf sb) {
  const int4 blk = d.gblk[blockIdx.x];
  const int inst = blk.x;
  const InstParams& P = d.prm[inst];
  Clock& C = d.clk[inst];
  const int t = threadIdx.x;
  const bool is_ghost = t < blk.z;
  const int g = blk.y + t;
  const bool disk = blk.w == 1;
  float vmag = 0.0f;
  float fx = 0.0f;
  if (is_ghost) {
    const uint32_t s = d.gslot[P.gmap0 + g];
    const uint32_t K = sb.cell[s];
    const float4 pg = sb.pv[s];
    const Shep S = shepard(d, P, sb, K, pg.x, pg.y);
    const float vwx = disk ? (float)C.vd : 0.0f;
    const float awx = disk ? (float)C.ad : 0.0f;
    float p, vgx, vgy;
    if (S.W > 0.0f) {
      const float inv = 1.0f / S.W;
      // body-force term (g - a_w) . sum rho_j (r_g - r_j) W
      p = (S.p + (0.0f - awx) * S.rx + P.gy * S.ry) * inv;
      vgx = 2.0f * vwx - S.vx * inv;
      vgy = -S.vy * inv;
    } else {
      p = 0.0f;
      vgx = vwx;
      vgy = 0.0f;
    }
    p = fmaxf(p, P.p_cav);
    float rg;
    if (P.ghost_rho_mode == 0) rg = P.rho0 * (1.0f + p * P.inv_rho0c02);
    else rg = P.rho0 * expf(P.inv_gamma * log1pf(p / P.B));
    const float Pg = p / (rg * rg);
    const float cg = P.c0 * expf(P.c_exp * log1pf((rg - P.rho0) / P.rho0));
    const float m = disk ? P.m_disk : P.m_wall;
    sb.pv[s] = make_float4(pg.x, pg.y, vgx, vgy);
    sb.aux[s] = make_float4(rg, Pg, cg, -m);
    vmag = fast_sqrt(vgx * vgx + vgy * vgy);
    if (MODE == EV_B && disk) {
      // x force of this ring ghost on its fluid neighbours (pressure + AV)
      int cx, cy;
      cell_xy(P, K, cx, cy);
      for (int dy = -1; dy <= 1; ++dy) {
        const int yy = cy + dy;
        if (yy < 0 || yy >= P.ncy) continue;
        for (int dx = -1; dx <= 1; ++dx) {
          const int xx = cx + dx;
          if (xx < 0 || xx >= P.ncx) continue;
          const uint32_t K2 = (uint32_t)(P.cell_off + yy * P.ncx + xx);
          for (uint32_t j = d.start[K2]; j < d.start[K2 + 1]; ++j) {
            const float4 aj = sb.aux[j];
            if (!(aj.w > 0.0f)) continue;
            const float4 pj = sb.pv[j];
            const float rx = (pj.x + (float)dx * P.dc) - pg.x;  // r_i - r_g
            const float ry = (pj.y + (float)dy * P.dc) - pg.y;
            const float r2 = rx * rx + ry * ry;
            if (!(r2 < P.four_h2)) continue;
            float W, F;
            wendland(P, r2, W, F);
            const float vr = (pj.z - vgx) * rx + (pj.w - vgy) * ry;
            const float rsum = aj.x + rg, den = r2 + P.eta2h2;
            const float inv = fast_rcp(den * rsum);
            const float piav = vr < 0.0f ? -P.alpha * (aj.z + cg) * P.h * vr * inv : 0.0f;
            fx -= aj.w * m * (aj.y + Pg + piav) * F * rx;
          }
        }
      }
    }
  }
  if (MODE == EV_A) {
    if constexpr (BATCH) {
      if (is_ghost && vmag > 0.0f) atomicMax(&C.vmax_bits, __float_as_uint(vmag));
    } else {
      vmax_update<false>(d.clk, 0, is_ghost, vmag);
    }
    // probes: Shepard average of the fluid pressure at fixed wall points
    if (disk && t >= blk.z && t < blk.z + P.n_probes) {
      const int k = t - blk.z;
      const Shep S = shepard(d, P, sb, P.probe_cell[k], P.probe_ox[k], P.probe_oy[k]);
      const float pk = S.W > 0.0f ? S.p / S.W : 0.0f;
      const long long row = (long long)inst * WC_HIST_CAP + (C.step % WC_HIST_CAP);
      d.hist_p[row * WC_MAX_PROBES + k] = pk;
    }
  }
  if (MODE == EV_B && disk) {
    // fixed-order block reduction of the ring force, FP64
    __shared__ double ws[WC_GHOST_BLOCK / 64];
    const double v = wave_sum((double)fx);
    if ((t & 63) == 0) ws[t >> 6] = v;
    __syncthreads();
    if (t == 0) {
      double f = 0.0;
      for (int w = 0; w < WC_GHOST_BLOCK / 64; ++w) f += ws[w];
      C.w_boundary += C.dt * f * C.vd;
    }
  }
}

// Pair sums + predictor (eval A) / corrector (eval B) for every fluid slot;
// ghost slots are carried into the output buffer. EV_EXPORT writes the rates.
template <int MODE, bool BATCH>
__global__ __launch_bounds__(WC_BLOCK) void k_pair(Dev d, Buf sb, Buf base, Buf out) {
  const int s = xcd_block(blockIdx.x, gridDim.x) * WC_BLOCK + threadIdx.x;
  const bool inr = s < d.n_slots;
  const int inst = inr ? inst_at<BATCH>(sb, s) : 0;
  const InstParams& P = d.prm[inst];
  Clock* clk = d.clk;
  const Clock& C = clk[inst];
  uint32_t K = 0;
  float4 pi = make_float4(0, 0, 0, 0), ai = make_float4(0, 0, 0, 0);
  if (inr) {
    K = sb.cell[s];
    pi = sb.pv[s];
    ai = sb.aux[s];
  }
  const bool fluid = inr && ai.w > 0.0f;
  if (MODE == EV_A && inr && !fluid) {
    out.cell[s] = K;
    out.id[s] = sb.id[s];
    out.pv[s] = pi;
    out.aux[s] = make_float4(ai.x, 0.0f, 0.0f, 0.0f);
    if constexpr (BATCH) out.inst[s] = (uint16_t)inst;
  }
  PairAcc acc = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
  if (fluid) pair_sums(d, P, sb, s, K, pi, ai, acc);
  if (MODE == EV_EXPORT) {
    if (fluid) {
      d.xr[s] = acc.D;
      d.xr[d.n_slots + s] = acc.ax;
      d.xr[2 * d.n_slots + s] = acc.ay + P.gy;
      d.xr[3 * d.n_slots + s] = pi.z + acc.Vx;
      d.xr[4 * d.n_slots + s] = pi.w + acc.Vy;
    }
    return;
  }
  bool clamp_hit = false, enf_hit = false;
  float vnew = 0.0f;
  if (fluid) {
    const double dt = MODE == EV_A ? step_dt(d, P, C) : C.dt;
    const float hdt = (float)(MODE == EV_A ? 0.5 * dt : dt);
    const double te = C.t + (MODE == EV_A ? 0.5 * dt : dt);
    uint32_t Kb;
    float4 pb;
    float rb;
    if (MODE == EV_A) {
      Kb = K;
      pb = pi;
      rb = ai.x;
    } else {
      Kb = base.cell[s];
      pb = base.pv[s];
      rb = base.aux[s].x;
    }
    float rn = rb + hdt * acc.D;
    if (rn < P.rho_lo) { rn = P.rho_lo; clamp_hit = true; }
    if (rn > P.rho_hi) { rn = P.rho_hi; clamp_hit = true; }
    float vx = pb.z + hdt * acc.ax;
    float vy = pb.w + hdt * (acc.ay + P.gy);
    float ox = pb.x + hdt * (pi.z + acc.Vx);
    float oy = pb.y + hdt * (pi.w + acc.Vy);
    int cx, cy;
    cell_xy(P, Kb, cx, cy);
    renorm(ox, cx, P.dc);
    renorm(oy, cy, P.dc);
    // enforcement in FP64: hard walls, then radial pull-out from the disk
    double x = P.x_lo + (double)cx * P.dcd + (double)ox;
    double y = P.y_lo + (double)cy * P.dcd + (double)oy;
    bool moved = false;
    const double e = P.eps_wall;
    if (x < e) { x = e; vx = -vx; moved = true; }
    if (x > P.L - e) { x = P.L - e; vx = -vx; moved = true; }
    if (y < e) { y = e; vy = -vy; moved = true; }
    if (y > P.W - e) { y = P.W - e; vy = -vy; moved = true; }
    if (P.nd > 0) {
      double xd, vd, ad;
      kinematics(P, te, xd, vd, ad);
      const double rx = x - xd, ry = y - P.disk_y0;
      const double d2 = rx * rx + ry * ry;
      if (d2 < P.R * P.R) {
        double nx = -1.0, ny = 0.0;
        if (d2 > 0.0) {
          const double dd = sqrt(d2);
          nx = rx / dd;
          ny = ry / dd;
        }
        x = xd + (P.R + e) * nx;
        y = P.disk_y0 + (P.R + e) * ny;
        const double w = ((double)vx - vd) * nx + (double)vy * ny;
        if (w < 0.0) {
          vx = (float)((double)vx - 2.0 * w * nx);
          vy = (float)((double)vy - 2.0 * w * ny);
        }
        moved = true;
      }
    }
    enf_hit = moved;
    if (moved) {
      encode_axis(x, P.x_lo, P.dcd, P.dc, P.ncx, cx, ox);
      encode_axis(y, P.y_lo, P.dcd, P.dc, P.ncy, cy, oy);
    }
    cx = min(max(cx, 0), P.ncx - 1);
    cy = min(max(cy, 0), P.ncy - 1);
    const uint32_t Kn = (uint32_t)(P.cell_off + cy * P.ncx + cx);
    out.cell[s] = Kn;
    out.pv[s] = make_float4(ox, oy, vx, vy);
    out.aux[s] = make_float4(rn, 0.0f, 0.0f, 0.0f);
    if (MODE == EV_A) {
      out.id[s] = sb.id[s];
      if constexpr (BATCH) out.inst[s] = (uint16_t)inst;
    }
    out.bslot[s] = atomicAdd(&d.count[Kn], 1u);
    vnew = fast_sqrt(vx * vx + vy * vy);
    if (!(rn == rn) || !(vnew <= 3.0e38f)) atomicOr(&clk[inst].bad, 1u);
  }
  count_hits<BATCH>(clk, inst, clamp_hit, enf_hit);
  if (MODE == EV_B) {
    vmax_update<BATCH>(clk, inst, fluid, vnew);
    if (blockIdx.x == 0 && threadIdx.x < d.n_inst) {
      Clock& Ci = clk[threadIdx.x];
      Ci.t_next = Ci.t + Ci.dt;
    }
  }
}

// First bucket slots and v_max of a freshly loaded state (slots in any order).
template <bool BATCH>
__global__ __launch_bounds__(WC_BLOCK) void k_init(Dev d, Buf X) {
  const int s = blockIdx.x * WC_BLOCK + threadIdx.x;
  const bool inr = s < d.n_slots;
  const int inst = inr ? inst_at<BATCH>(X, s) : 0;
  const InstParams& P = d.prm[inst];
  bool fl = false;
  float v = 0.0f;
  if (inr) {
    const int local = (int)X.id[s] - P.id0;
    fl = local < P.nf;
    if (fl) {
      X.bslot[s] = atomicAdd(&d.count[X.cell[s]], 1u);
      const float4 pv = X.pv[s];
      v = fast_sqrt(pv.z * pv.z + pv.w * pv.w);
    }
  }
  vmax_update<BATCH>(d.clk, inst, fl, v);
}

// FP64 diagnostics of every instance; one block per instance, fixed order.
__global__ __launch_bounds__(1024) void k_diag(Dev d, Buf X, int row, int sorted) {
  const int i = blockIdx.x;
  const InstParams& P = d.prm[i];
  Clock& C = d.clk[i];
  int lo, hi;
  if (sorted) {
    lo = (int)d.start[P.cell_off];
    hi = (int)d.start[P.cell_off + P.ncell];
  } else {
    lo = P.id0;
    hi = P.id0 + P.nf + P.nw + P.nd;
  }
  double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};  // M, Px, Py, KE, Eel, Epot, ncav, bad
  const double g = P.gammad, r0 = P.rho0d, B = P.Bd;
  const double rc = r0 * pow(1.0 + P.p_cavd / B, 1.0 / g);
  auto e_tait = [&](double q) {
    return B * ((pow(q, g - 1.0) - pow(r0, g - 1.0)) / ((g - 1.0) * pow(r0, g)) + 1.0 / q - 1.0 / r0);
  };
  const double erc = e_tait(rc);
  const double m = P.m_fluidd;
  for (int s = lo + (int)threadIdx.x; s < hi; s += 1024) {
    const int local = (int)X.id[s] - P.id0;
    if (local < 0 || local >= P.nf) continue;
    const float4 pv = X.pv[s];
    const double r = (double)X.aux[s].x;
    int cx, cy;
    cell_xy(P, X.cell[s], cx, cy);
    const double y = P.y_lo + (double)cy * P.dcd + (double)pv.y;
    const double u = pv.z, w = pv.w;
    acc[0] += m;
    acc[1] += m * u;
    acc[2] += m * w;
    acc[3] += 0.5 * m * (u * u + w * w);
    acc[4] += m * (r >= rc ? e_tait(r) : erc + P.p_cavd * (1.0 / rc - 1.0 / r));
    acc[5] += m * (-(double)P.gy) * y;
    acc[6] += (B * (pow(r / r0, g) - 1.0) <= P.p_cavd) ? 1.0 : 0.0;
    if (!(r == r) || !(fabs(u) < 1e30) || !(fabs(w) < 1e30)) acc[7] += 1.0;
  }
  __shared__ double ws[16][8];
  for (int k = 0; k < 8; ++k) {
    const double v = wave_sum(acc[k]);
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6][k] = v;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double tot[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int w = 0; w < 16; ++w)
      for (int k = 0; k < 8; ++k) tot[k] += ws[w][k];
    double xd, vd, ad;
    kinematics(P, C.t_next, xd, vd, ad);
    double* o = d.diag + ((long long)i * WC_DIAG_CAP + (row % WC_DIAG_CAP)) * WC_NDIAG;
    o[0] = C.t_next;
    o[1] = C.step >= 0 ? C.dt : 0.0;
    o[2] = C.step >= 0 ? C.vmax_used : 0.0;
    o[3] = tot[0];
    o[4] = tot[1];
    o[5] = tot[2];
    o[6] = tot[3];
    o[7] = tot[4];
    o[8] = tot[5];
    o[9] = 0.5 * P.disk_mass * vd * vd;
    o[10] = C.w_boundary;
    o[11] = (double)(C.step + 1);
    o[12] = (double)C.n_clamp;
    o[13] = tot[6];
    o[14] = (double)C.n_enforce;
    if (tot[7] > 0.0 || !(tot[3] == tot[3])) C.bad |= 1u;
  }
}

// Test hook: in-support neighbour count and id sum per sorted slot.
__global__ __launch_bounds__(WC_BLOCK) void k_neigh(Dev d, Buf sb) {
  const int s = blockIdx.x * WC_BLOCK + threadIdx.x;
  if (s >= d.n_slots) return;
  const InstParams& P = d.prm[0];
  const uint32_t K = sb.cell[s];
  const float4 pi = sb.pv[s];
  int cx, cy;
  cell_xy(P, K, cx, cy);
  int n = 0;
  long long sum = 0;
  for (int dy = -1; dy <= 1; ++dy) {
    const int yy = cy + dy;
    if (yy < 0 || yy >= P.ncy) continue;
    for (int dx = -1; dx <= 1; ++dx) {
      const int xx = cx + dx;
      if (xx < 0 || xx >= P.ncx) continue;
      const uint32_t K2 = (uint32_t)(P.cell_off + yy * P.ncx + xx);
      for (uint32_t j = d.start[K2]; j < d.start[K2 + 1]; ++j) {
        if (j == (uint32_t)s) continue;
        const float4 pj = sb.pv[j];
        const float rx = (pi.x - pj.x) - (float)dx * P.dc;
        const float ry = (pi.y - pj.y) - (float)dy * P.dc;
        if (rx * rx + ry * ry < P.four_h2) {
          ++n;
          sum += (long long)sb.id[j];
        }
      }
    }
  }
  d.nb_count[s] = n;
  d.nb_idsum[s] = sum;
}

// ---------------------------------------------------------------------------
// Launch wrappers (host side of this translation unit).

#define NB(n) (((n) + WC_BLOCK - 1) / WC_BLOCK)

template <bool BATCH>
static void eval_sort(const Dev& d, hipStream_t st, int mode, const Buf& pre, const Buf& out,
                      const Buf& pre2, const Buf& out2) {
  const int nb = NB(d.n_slots);
  if (mode == EV_A) k_kin<EV_A><<<d.n_inst, 256, 0, st>>>(d, pre);
  else if (mode == EV_B) k_kin<EV_B><<<d.n_inst, 256, 0, st>>>(d, pre);
  else k_kin<EV_EXPORT><<<d.n_inst, 256, 0, st>>>(d, pre);
  k_scan<<<1, 1024, 0, st>>>(d);
  k_scatter<BATCH><<<nb, WC_BLOCK, 0, st>>>(d, pre);
  if (mode == EV_B) k_permute<EV_B, BATCH><<<nb, WC_BLOCK, 0, st>>>(d, pre, out, pre2, out2);
  else k_permute<EV_A, BATCH><<<nb, WC_BLOCK, 0, st>>>(d, pre, out, pre2, out2);
}

template <bool BATCH>
static void enqueue_step_t(const Dev& d, const Bufs& b, int n_gblk, hipStream_t st) {
  const int nb = NB(d.n_slots);
  eval_sort<BATCH>(d, st, EV_A, b.X, b.Y, b.Y, b.Y);
  k_ghost<EV_A, BATCH><<<n_gblk, WC_GHOST_BLOCK, 0, st>>>(d, b.Y);
  k_pair<EV_A, BATCH><<<nb, WC_BLOCK, 0, st>>>(d, b.Y, b.Y, b.Z);
  eval_sort<BATCH>(d, st, EV_B, b.Z, b.W, b.Y, b.X);
  k_ghost<EV_B, BATCH><<<n_gblk, WC_GHOST_BLOCK, 0, st>>>(d, b.W);
  k_pair<EV_B, BATCH><<<nb, WC_BLOCK, 0, st>>>(d, b.W, b.X, b.X);
}

void wc_enqueue_step(const Dev& d, const Bufs& b, int n_gblk, bool batch, hipStream_t st) {
  if (batch) enqueue_step_t<true>(d, b, n_gblk, st);
  else enqueue_step_t<false>(d, b, n_gblk, st);
}

void wc_enqueue_init(const Dev& d, const Bufs& b, bool batch, hipStream_t st) {
  if (batch) k_init<true><<<NB(d.n_slots), WC_BLOCK, 0, st>>>(d, b.X);
  else k_init<false><<<NB(d.n_slots), WC_BLOCK, 0, st>>>(d, b.X);
}

void wc_enqueue_diag(const Dev& d, const Bufs& b, int row, bool sorted, hipStream_t st) {
  k_diag<<<d.n_inst, 1024, 0, st>>>(d, b.X, row, sorted ? 1 : 0);
}

// Eval-A sort of X into Y without advancing the clock (test hooks).
void wc_enqueue_export_sort(const Dev& d, const Bufs& b, bool batch, hipStream_t st) {
  if (batch) eval_sort<true>(d, st, EV_EXPORT, b.X, b.Y, b.Y, b.Y);
  else eval_sort<false>(d, st, EV_EXPORT, b.X, b.Y, b.Y, b.Y);
}

void wc_enqueue_export_ghosts(const Dev& d, const Bufs& b, int n_gblk, hipStream_t st) {
  k_ghost<EV_EXPORT, false><<<n_gblk, WC_GHOST_BLOCK, 0, st>>>(d, b.Y);
}

void wc_enqueue_export_pair(const Dev& d, const Bufs& b, hipStream_t st) {
  k_pair<EV_EXPORT, false><<<NB(d.n_slots), WC_BLOCK, 0, st>>>(d, b.Y, b.Y, b.Z);
}

void wc_enqueue_pair_a(const Dev& d, const Bufs& b, bool batch, hipStream_t st) {
  if (batch) k_pair<EV_A, true><<<NB(d.n_slots), WC_BLOCK, 0, st>>>(d, b.Y, b.Y, b.Z);
  else k_pair<EV_A, false><<<NB(d.n_slots), WC_BLOCK, 0, st>>>(d, b.Y, b.Y, b.Z);
}

void wc_enqueue_neigh(const Dev& d, const Bufs& b, hipStream_t st) {
  k_neigh<<<NB(d.n_slots), WC_BLOCK, 0, st>>>(d, b.Y);
}
