// wcsph_kernels.hip -- HIP kernels of the planar WCSPH step for gfx950.
//
// One step = two evaluations (predictor-corrector). Each evaluation runs:
//   k_sort     the cell list: stable counting sort of the slots by cell key
//              from the cell buckets (per-tile entry totals -> cell
//              ranges, buckets ordered by old slot, gather into sorted
//              order, per-particle EOS P = p/rho^2 and c); its first block
//              advances the clock and the prescribed disk kinematics
//   k_ghost    Adami-Shepard ghost state on walls and ring, probes (eval A),
//              v_max of the ghosts (eval A), work of the ring (eval B)
//   k_pair     pair sums over the 3x3 cells (continuity + delta, pressure +
//              AV + laminar, XSPH) fused with the predictor / corrector,
//              density band, enforcement, new cell key; every slot goes
//              into the bucket of its cell for the next sort, the disk ring
//              placed at the next evaluation's time
// Pair arithmetic is FP32 on cell-relative offsets; time, kinematics,
// enforcement geometry and diagnostics are FP64.

#include "wcsph_launch.h"
#include "wcsph_kin.h"

// Scan shapes of the pair pass (UCAP, LCAP, RU) picked for this GPU by the
// autotuner (paper_2609_05494_amd/autotune.py), when it has been run; the
// defaults below otherwise. They change speed only: every shape sums each
// particle's pairs in the same order.
#if __has_include("wcsph_tuned.h")
#include "wcsph_tuned.h"
#endif

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

// Disk state at time te of the current step: a coupled disk is extrapolated
// from its state at t with its latest acceleration, otherwise the prescribed
// law.
__device__ void disk_at(const InstParams& P, const Clock& C, double te, double& x, double& v, double& a) {
  if (P.kin_mode == 2 && C.coupled) {
    const double tau = te - C.t;
    x = C.xc + tau * C.vc;
    v = C.vc + tau * C.ac;
    a = C.ac;
  } else {
    kinematics(P, te, x, v, a);
  }
}

// Disk state of the newest particle state (time t_next).
__device__ void disk_newest(const InstParams& P, const Clock& C, double& x, double& v, double& a) {
  if (P.kin_mode == 2 && C.coupled) {
    x = C.xd_next;
    v = C.vd_next;
    a = C.ac_next;
  } else {
    kinematics(P, C.t_next, x, v, a);
  }
}

// Tait pressure with the cavitation cutoff, P = p / rho^2 and the sound speed
// c0 (rho/rho0)^((gamma-1)/2), with x = rho/rho0 - 1 so that p stays accurate
// near rho0 in FP32. For gamma = 7, (1 + x)^7 - 1 is x times its binomial
// polynomial and the sound speed exponent is 3; otherwise log1p/expm1.
// The Mie-Grueneisen law at zero internal energy (eos_type 1) at
// mu = rho/rho0 - 1: capped at mu_max; K mu (1 + k1 mu) / (1 - b mu)^2 and
// c = C sqrt((1 + (2 k1 + b) mu) / (1 - b mu)^3) in compression, K mu and C
// in tension (before the cutoff).
__device__ __forceinline__ void mg_eos(const InstParams& P, float x, float& p, float& c) {
  const float mu = fminf(x, P.mg_mu_max);
  if (mu >= 0.0f) {
    const float den = 1.0f - P.mg_b * mu, iden = 1.0f / den;
    p = P.mg_K * mu * (1.0f + P.mg_k1 * mu) * (iden * iden);
    c = P.c0 * sqrtf((1.0f + (2.0f * P.mg_k1 + P.mg_b) * mu) * (iden * iden * iden));
  } else {
    p = P.mg_K * mu;
    c = P.c0;
  }
}

// MG: some instance uses the Mie-Grueneisen law (else the check is compiled out).
// e: the specific internal energy (scheme 1; 0 otherwise), which adds the
// energy term of eq. eos to the Mie-Grueneisen pressure, (gamma0 + a mu)
// rho0 (1 + mu) e at the capped mu in compression, gamma0 rho e in tension.
template <bool MG>
__device__ __forceinline__ void fluid_eos(const InstParams& P, float rho, float& Pq, float& c, float e = 0.0f) {
  const float x = (rho - P.rho0) / P.rho0;
  float p;
  if (MG && P.eos_type == 1) {
    mg_eos(P, x, p, c);
    const float mu = fminf(x, P.mg_mu_max);
    p += (mu >= 0.0f ? P.mg_g0 + P.mg_a * mu : P.mg_g0) * (P.rho0 * (1.0f + mu)) * e;
  } else if (P.gamma == 7.0f) {
    const float y = 1.0f + x;
    p = P.B * (x * (7.0f + x * (21.0f + x * (35.0f + x * (35.0f + x * (21.0f + x * (7.0f + x)))))));
    c = P.c0 * (y * y * y);
  } else {
    const float l = log1pf(x);
    p = P.B * expm1f(P.gamma * l);
    c = P.c0 * expf(P.c_exp * l);
  }
  p = fmaxf(p, P.p_cav);
  Pq = p / (rho * rho);
}

// Wendland C2 (2D): W = sigma (1-q/2)^4 (2q+1); grad_i W = F r_ij,
// F = -fgrad (1-q/2)^3.
template <class PP>
__device__ __forceinline__ void wendland(const PP& P, float r2, float& W, float& F) {
  const float q = fast_sqrt(r2) * P.inv_h;
  const float s = 1.0f - 0.5f * q;
  const float s2 = s * s;
  W = P.sigma * s2 * s2 * (2.0f * q + 1.0f);
  F = -P.fgrad * s2 * s;
}

// Cubic B-spline of eq. cubic-kernel in 2D (the paper's kernel), sigma_c =
// 10 / (7 pi h^2): W = sigma_c (1 - 3/2 q^2 + 3/4 q^3) for q <= 1 and
// sigma_c (2 - q)^3 / 4 for 1 < q < 2; F = (1/r) dW/dr = (sigma_c / h^2)
// (9/4 q - 3) inside, -(3/4)(sigma_c / h^2)(2 - q)^2 / q outside.
template <class PP>
__device__ __forceinline__ void cubic_spline(const PP& P, float r2, float& W, float& F) {
  const float q = fast_sqrt(r2) * P.inv_h;
  const float s = 2.0f - q;
  const bool in = q <= 1.0f;
  const float w_in = P.kc_sigma * (1.0f + q * q * (0.75f * q - 1.5f));
  const float f_in = P.kc_a * (2.25f * q - 3.0f);
  const float w_out = 0.25f * P.kc_sigma * s * s * s;
  const float f_out = -0.75f * P.kc_a * s * s * fast_rcp(in ? 1.0f : q);
  W = in ? w_in : w_out;
  F = in ? f_in : f_out;
}


// Element j of a slot array through a 32-bit byte offset (the library
// keeps j * 16 below 2^32), so that the load is a scalar base plus one
// 32-bit lane offset rather than a 64-bit address per lane.
template <class T>
__device__ __forceinline__ T at32(const T* base, uint32_t j) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + j * (uint32_t)sizeof(T));
}


__device__ __forceinline__ void cell_xy(const InstParams& P, uint32_t K, int& cx, int& cy) {
  const int local = (int)K - P.cell_off;
  cy = local / P.ncx;
  cx = local - cy * P.ncx;
}

// Encode an FP64 position into (cell, FP32 offset inside the cell): the
// cell from u / dc (by the inverse edge, then corrected so that the offset
// lies in [0, dc)), clamped to the grid.
__device__ __forceinline__ void encode_axis(double x, double lo, double dcd, double inv_dcd, float dc, int n,
                                            int& c, float& o) {
  const double u = x - lo;
  double cf = floor(u * inv_dcd);
  double r = u - cf * dcd;
  if (r < 0.0) {
    cf -= 1.0;
    r += dcd;
  } else if (r >= dcd) {
    cf += 1.0;
    r -= dcd;
  }
  c = (int)fmin(fmax(cf, 0.0), (double)(n - 1));
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

// dt of the current step: the fixed table where it covers the step, else the
// CFL gate of eq. cfl from v_max (float bits vb).
__device__ __forceinline__ double step_dt_bits(const Dev& d, const InstParams& P, const Clock& C,
                                               unsigned int vb) {
  if (d.n_dt > 0) {
    const long long k = C.step - d.dt_step0;
    if (k >= 0 && k < d.n_dt) return d.dt_table[k];
  }
  const float vm = __uint_as_float(vb);
  return P.cfl * P.hd / (P.c0d + (double)vm);
}
__device__ __forceinline__ double step_dt(const Dev& d, const InstParams& P, const Clock& C) {
  return step_dt_bits(d, P, C, C.vmax_bits);
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
// wave holds a single instance, else one per lane. The stored value only
// grows during a kernel, so a wave whose maximum does not exceed the value
// it reads skips the atomic (this keeps thousands of waves from
// serialising on one address).
__device__ __forceinline__ void vmax_atomic(unsigned int* a, float w) {
  if (w > 0.0f && __float_as_uint(w) > __atomic_load_n(a, __ATOMIC_RELAXED)) atomicMax(a, __float_as_uint(w));
}
template <bool BATCH>
__device__ __forceinline__ void vmax_update(Clock* clk, int inst, bool act, float v) {
  const float m = act ? v : 0.0f;
  if constexpr (BATCH) {
    const int i0 = __shfl(inst, 0);
    if (__all(inst == i0)) {
      const float w = wave_max(m);
      if ((threadIdx.x & 63) == 0) vmax_atomic(&clk[i0].vmax_bits, w);
    } else if (act) {
      vmax_atomic(&clk[inst].vmax_bits, m);
    }
  } else {
    const float w = wave_max(m);
    if ((threadIdx.x & 63) == 0) vmax_atomic(&clk[0].vmax_bits, w);
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

// Energy audit sums of a fluid particle (second evaluation, audit runs):
// per unit mass of the particle, the dissipation of the artificial and
// laminar viscosity of its fluid pairs (half of each pair term), the delta
// term of its density rate (times P_i afterwards) and the fluid energy rate
// of its ghost pairs.
struct AudAcc {
  float av, visc, del, ghost;
};

// One of the three cell rows around (cx, cy): slots [rs, re) of its (up to)
// three cells, middle cell [ms, me).
struct RowRange {
  uint32_t rs, ms, me, re;
};
__device__ __forceinline__ RowRange row_range(const Dev& d, const InstParams& P, int cx, int cy, int dy) {
  RowRange r = {0u, 0u, 0u, 0u};
  const int yy = cy + dy;
  if (yy < 0 || yy >= P.ncy) return r;
  const int xlo = max(cx - 1, 0), xhi = min(cx + 1, P.ncx - 1);
  const uint32_t k0 = (uint32_t)(P.cell_off + yy * P.ncx);
  r.rs = at32(d.start, k0 + (uint32_t)xlo);
  r.ms = at32(d.start, k0 + (uint32_t)cx);
  r.me = at32(d.start, k0 + (uint32_t)cx + 1u);
  r.re = at32(d.start, k0 + (uint32_t)xhi + 1u);
  return r;
}
// cell shift code of slot j inside a row: 0 left, 1 middle, 2 right
__device__ __forceinline__ uint32_t dx_code(uint32_t j, const RowRange& r) {
  return j < r.ms ? 0u : (j < r.me ? 1u : 2u);
}

// Pair law of fluid particle i (state pi, rho_i, P_i = p_i/rho_i^2, c_i) with
// neighbour j at r_ij = (rx, ry): continuity + delta diffusion, pressure + AV
// (symmetric form), laminar (Lo-Shao), XSPH. Branch-free: a ghost neighbour
// (m < 0) contributes nothing to the delta and XSPH terms through m_fl = 0,
// and the AV switch is min(v_ij . r_ij, 0).
// VAR: bit 0 the quadratic AV term, bit 1 the cubic spline kernel, bit 2
// (scheme 1) D takes the internal-energy rate (1/2) m_j Pi_ij F v_ij . r_ij
// instead of the continuity and delta terms, bit 3 (scheme 1 density pass)
// D takes m_j W_ij and nothing else is summed.
template <bool AUD, int VAR, class PP>
__device__ __forceinline__ void pair_body(const PP& P, const float4& pi, float rhoi, float Pi,
                                          float ci, float rx, float ry, float r2, const float4& pj,
                                          const float4& aj, PairAcc& acc, AudAcc& aud) {
  float W, F;
  if constexpr ((VAR & 2) != 0) cubic_spline(P, r2, W, F);
  else wendland(P, r2, W, F);
  if constexpr ((VAR & 8) != 0) {  // summation density: |m_j| W_ij over fluid and ghosts
    acc.D += fabsf(aj.w) * W;
    return;
  }
  const float vxij = pi.z - pj.z, vyij = pi.w - pj.w;
  const float vr = vxij * rx + vyij * ry;
  const float mj = fabsf(aj.w);
  const float mfl2 = aj.w + mj;  // 2 m_j for fluid, 0 for ghosts (the halves below are exact)
  const float rsum = rhoi + aj.x;       // 2 rho_bar
  const float den = r2 + P.eta2h2;      // r^2 + eta^2 h^2
  const float inv = fast_rcp(den * rsum);
  // Monaghan AV: -alpha c_bar mu / rho_bar = -alpha (c_i + c_j) h vr inv for vr < 0
  const float vrm = fminf(vr, 0.0f);
  float piav = -P.alpha * P.h * (ci + aj.z) * vrm * inv;
  // quadratic term beta mu^2 / rho_bar = 2 beta h^2 vr^2 / ((r^2 + eta^2 h^2)^2 2 rho_bar)
  if constexpr ((VAR & 1) != 0) piav += P.beta2h2 * vrm * vrm * inv * (rsum * inv);
  const float mF = mj * F;
  // continuity + delta diffusion 2 delta h c0 (m_j / rho_j)(rho_i - rho_j) F (fluid pairs)
  const float dd = (0.5f * P.two_delta_h_c0) * mfl2 * fast_rcp(aj.x) * (rhoi - aj.x) * F;
  if constexpr ((VAR & 4) != 0) acc.D += 0.5f * mF * piav * vr;
  else acc.D += mF * vr + dd;
  const float sp = Pi + aj.y + piav;
  // laminar (Lo-Shao): 4 nu0 m_j F r^2 / ((rho_i + rho_j)(r^2 + eta^2 h^2)) v_ij
  const float lam = P.four_nu0 * mF * r2 * inv;
  acc.ax += lam * vxij - mF * sp * rx;
  acc.ay += lam * vyij - mF * sp * ry;
  if constexpr (AUD) {
    // fluid pairs: the pressure work cancels the elastic energy rate of the
    // continuity term pair by pair; half of each viscous dissipation
    // (1/2) m_j Pi_ij F v_ij.r_ij and -(1/2) lam |v_ij|^2 (F < 0), and the
    // delta term. Ghost pairs whole: the work of the pair's pressure, AV and
    // laminar forces on v_i plus P_i m_g F v_ig.r_ig of the continuity term,
    // -m_g F ((P_g + Pi_ig) r.v_i + P_i r.v_g) + lam v_ig.v_i.
    const float mflF = 0.5f * mfl2 * F, mgF = mF - mflF;
    const float v2 = vxij * vxij + vyij * vyij;
    const float lamg = P.four_nu0 * mgF * r2 * inv;
    aud.av += 0.5f * mflF * piav * vr;
    aud.visc -= 0.5f * (lam - lamg) * v2;
    aud.del += dd;
    aud.ghost += lamg * (vxij * pi.z + vyij * pi.w) -
                 mgF * ((aj.y + piav) * (rx * pi.z + ry * pi.w) + Pi * (rx * pj.z + ry * pj.w));
  }
  // XSPH eps (m_j / rho_bar) W (v_j - v_i) over fluid; 1 / rho_bar = 2 den inv
  const float w = P.eps_xsph * mfl2 * den * inv * W;
  acc.Vx -= w * vxij;
  acc.Vy -= w * vyij;
}

#ifndef PAIR_G
#define PAIR_G 4                        // lanes per slot in the pair sums
#endif
#define PAIR_SLOTS 64                   // slots per block
#define PAIR_BLOCK (PAIR_SLOTS * PAIR_G)
#define SCAN_UNROLL 4

// Fixed-order sum over the PAIR_G lanes of a slot (xor butterfly: the same
// bits on every lane of the group).
__device__ __forceinline__ float slot_sum(float v) {
  for (int o = 1; o < PAIR_G; o <<= 1) v += __shfl_xor(v, o);
  return v;
}

// The parameters of the candidate test and the pair law, held in registers
// (the list stores below would otherwise force them to be reloaded).
struct PairC {
  float dc, four_h2, inv_h, sigma, fgrad, alpha, h, eta2h2, two_delta_h_c0, four_nu0, eps_xsph, beta2h2;
  float kc_sigma, kc_a;
};
__device__ __forceinline__ PairC pair_c(const InstParams& P) {
  PairC c;
  c.dc = P.dc;
  c.four_h2 = P.four_h2;
  c.inv_h = P.inv_h;
  c.sigma = P.sigma;
  c.fgrad = P.fgrad;
  c.alpha = P.alpha;
  c.h = P.h;
  c.eta2h2 = P.eta2h2;
  c.two_delta_h_c0 = P.two_delta_h_c0;
  c.four_nu0 = P.four_nu0;
  c.eps_xsph = P.eps_xsph;
  c.beta2h2 = P.beta2h2;
  c.kc_sigma = P.kc_sigma;
  c.kc_a = P.kc_a;
  return c;
}

#ifndef UCAP
#define UCAP 192  // union candidates staged per pass (one wave)
#endif
#ifndef LCAP
#define LCAP 16   // entries of a lane's hit list
#endif
#ifndef RU
#define RU 2      // unroll of a lane's walk along one of its rows
#endif
#define PAIR_STR2(x) #x
#define PAIR_STR(x) PAIR_STR2(x)

// Order the wave's LDS accesses: stores before this point are seen by every
// lane's loads after it (accesses of one wave are performed in order; the
// fences keep the compiler from moving them across).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Pair sums of the fluid slots of one wave (64 / PAIR_G consecutive slots,
// PAIR_G lanes each; every lane of the wave calls this). Fluid slots of one
// instance and one cell row form a group; the union of their 3x3 blocks is
// one slot range per row, which the wave stages in LDS in passes of UCAP entries:
// offset x, offset y seen from the group's row, cell column, slot. Each
// lane then walks its own particle's three rows of candidates (rows bottom
// to top; in each row, the row's cells left to right in sorted order, entry
// q, q + PAIR_G, ... for lane q) through LDS, keeps the in-support ones in a
// lane-private list and sums the pair law over the list. A lane's candidate
// order and every operand of a pair depend on the particle and its
// neighbours only, not on the other slots of the wave.
// EXP (export hook, single instance): every in-support neighbour's id also
// goes to the export buffer d.nb_ids by fluid index f: the count at [f]
// (zeroed by the host), the ids at [nf + f * WC_NB_CAP + k].
template <bool BATCH, bool AUD, int VAR, bool EXP = false>
__device__ __forceinline__ void pair_sums_wave(const Dev& d, const Buf& sb, int s, int inst, uint32_t K,
                                               bool fluid, float4 pi, float4 ai, int q, float4* U,
                                               uint8_t* my, PairAcc& acc, AudAcc& aud) {
  const InstParams& IP = d.prm[inst];
  const PairC P = pair_c(IP);
  const float rhoi = ai.x, Pi = ai.y, ci = ai.z;
  const uint32_t lane = threadIdx.x & 63u;
  int cx = 0, cy = 0;
  if (fluid) cell_xy(IP, K, cx, cy);
  // a single instance's grid, read once (the wave fences in the loop below
  // keep the compiler from hoisting these loads out of it)
  const int incx = IP.ncx, incy = IP.ncy, ioff = IP.cell_off;
  const float idc = IP.dc;
  uint64_t pending = __ballot(fluid);
  while (pending) {
    const int L = __builtin_ctzll(pending);
    const int ginst = __builtin_amdgcn_readlane(inst, L);
    const int gcy = __builtin_amdgcn_readlane(cy, L);
    const bool mem = fluid && inst == ginst && cy == gcy;
    const uint64_t mb = __ballot(mem);
    pending &= ~mb;
    const int cxa = __builtin_amdgcn_readlane(cx, L);
    const int cxb = __builtin_amdgcn_readlane(cx, 63 - __builtin_clzll(mb));
    const int gncx = BATCH ? d.prm[ginst].ncx : incx, gncy = BATCH ? d.prm[ginst].ncy : incy,
              goff = BATCH ? d.prm[ginst].cell_off : ioff;
    const float gdc = BATCH ? d.prm[ginst].dc : idc;
    // union rows: first slot, first cell key; union index bases ub1, ub2.
    // The cell-start loads of the union's rows complete together, then
    // those of the lane's own rows (the empty asm statements take them as
    // operands), without branches: a row outside the grid reads the nearest
    // row and its values are then replaced. Otherwise the compiler waits for
    // each row's loads before it issues the next row's.
    uint32_t va[3], vb[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      const int kc = goff + min(max(gcy + r - 1, 0), gncy - 1) * gncx;
      va[r] = at32(d.start, (uint32_t)(kc + max(cxa - 1, 0)));
      vb[r] = at32(d.start, (uint32_t)(kc + min(cxb + 1, gncx - 1) + 1));
    }
    asm("" : "+v"(va[0]), "+v"(va[1]), "+v"(va[2]), "+v"(vb[0]), "+v"(vb[1]), "+v"(vb[2]));
    uint32_t urs[3], un[3];
    int k0[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      const int yy = gcy + r - 1;
      const bool ok = yy >= 0 && yy < gncy;
      k0[r] = ok ? goff + yy * gncx : 0;
      urs[r] = ok ? __builtin_amdgcn_readfirstlane(va[r]) : 0u;
      un[r] = ok ? __builtin_amdgcn_readfirstlane(vb[r]) - __builtin_amdgcn_readfirstlane(va[r]) : 0u;
    }
    uint32_t ors[3], on[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      const int kc = goff + min(max(gcy + r - 1, 0), gncy - 1) * gncx;
      ors[r] = at32(d.start, (uint32_t)(kc + min(max(cx - 1, 0), gncx - 1)));  // (any lane's cx: clamped)
      on[r] = at32(d.start, (uint32_t)(kc + min(cx + 1, gncx - 1) + 1));
    }
    asm("" : "+v"(ors[0]), "+v"(ors[1]), "+v"(ors[2]), "+v"(on[0]), "+v"(on[1]), "+v"(on[2]));
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      on[r] = un[r] != 0u ? on[r] - ors[r] : 0u;
      ors[r] = un[r] != 0u ? ors[r] : 0u;
    }
    const uint32_t ub1 = un[0], ub2 = un[0] + un[1], n = ub2 + un[2];
    // own rows: candidate c of row r has union index c + adj[r]
    uint32_t p1 = 0u, p2 = 0u, no = 0u, adj0 = 0u, adj1 = 0u, adj2 = 0u;
    if (mem) {
      p1 = on[0];
      p2 = on[0] + on[1];
      no = p2 + on[2];
      adj0 = ors[0] - urs[0];
      adj1 = ub1 + (ors[1] - urs[1]) - p1;
      adj2 = ub2 + (ors[2] - urs[2]) - p2;
    }
    const float cxi = (float)(cx - cxa);
    int cnt = 0;
    // own row r is the union range [p_r + adj_r, p_r + adj_r + on_r); lane q
    // walks entries q, q + G, ... of each own row in turn (row, next union
    // index u, end of the row), carried from pass to pass
    int row = 0;
    uint32_t u = adj0 + (uint32_t)q, uend = adj0 + p1;
    // sum the pair law over the list, two entries in flight (buffers a, b)
    auto fetch = [&](int k, float4& E, float4& pj, float4& aj) __attribute__((always_inline)) {
      E = U[my[min(k, cnt - 1) * PAIR_BLOCK]];
      const uint32_t j = __float_as_uint(E.w);
      pj = at32(sb.pv, j);
      aj = at32(sb.aux, j);
    };
    auto body = [&](const float4& E, const float4& pj, const float4& aj) __attribute__((always_inline)) {
      const float rx = (pi.x - E.x) - (E.z - cxi) * P.dc;
      const float ry = pi.y - E.y;
      pair_body<AUD, VAR>(P, pi, rhoi, Pi, ci, rx, ry, rx * rx + ry * ry, pj, aj, acc, aud);
      if constexpr (EXP) {
        const uint32_t f = at32(sb.id, (uint32_t)s) - (uint32_t)IP.id0;
        const uint32_t k = atomicAdd(&d.nb_ids[f], 1u);
        if (k < (uint32_t)WC_NB_CAP)
          d.nb_ids[(size_t)IP.nf + (size_t)f * WC_NB_CAP + k] = at32(sb.id, __float_as_uint(E.w));
      }
    };
    auto flush = [&]() __attribute__((always_inline)) {
      if (cnt > 0) {
        float4 Ea, pa, aa, Eb, pb, ab;
        fetch(0, Ea, pa, aa);
        for (int k = 0;; k += 2) {
          fetch(k + 1, Eb, pb, ab);
          body(Ea, pa, aa);
          if (k + 1 >= cnt) break;
          fetch(k + 2, Ea, pa, aa);
          body(Eb, pb, ab);
          if (k + 2 >= cnt) break;
        }
      }
      cnt = 0;
    };
    for (uint32_t u0 = 0; u0 < n; u0 += UCAP) {
      const uint32_t m = min(n - u0, (uint32_t)UCAP);
      wave_sync();  // the previous pass is no longer read
      for (uint32_t t = lane; t < m; t += 64) {
        const uint32_t u = u0 + t;
        const bool a0 = u < ub1, a1 = u < ub2;
        const uint32_t j = a0 ? urs[0] + u : (a1 ? urs[1] + (u - ub1) : urs[2] + (u - ub2));
        const int kr = a0 ? k0[0] : (a1 ? k0[1] : k0[2]);
        const float sy = a0 ? -gdc : (a1 ? 0.0f : gdc);
        const float4 pj = at32(sb.pv, j);
        const int cxj = (int)at32(sb.cell, j) - kr;
        U[t] = make_float4(pj.x, pj.y + sy, (float)(cxj - cxa), __uint_as_float(j));
      }
      wave_sync();
      if (mem) {
        // a lane walks a row up to the nearer of the row's end, the pass's
        // end and the room left in its list; then it flushes the list, moves
        // to its next own row, or leaves the rest of the row to the next pass
        const uint32_t pe = u0 + m;
        for (;;) {
          const uint32_t lim = min(uend, pe);
          while (u < lim) {
            // the row's candidates in this pass, as many as the list has room for
            const uint32_t ue = u + PAIR_G * min((lim - u + PAIR_G - 1) / PAIR_G, (uint32_t)(LCAP - cnt));
            _Pragma(PAIR_STR(unroll RU))
            for (; u < ue; u += PAIR_G) {
              const float4 E = U[u - u0];
              const float rx = (pi.x - E.x) - (E.z - cxi) * P.dc;
              const float ry = pi.y - E.y;
              const bool hit = (rx * rx + ry * ry < P.four_h2) & (__float_as_uint(E.w) != (uint32_t)s);
              my[cnt * PAIR_BLOCK] = (uint8_t)(u - u0);
              cnt += hit ? 1 : 0;
            }
            if (cnt == LCAP) flush();
          }
          if (u < uend || row == 2) break;  // the pass ends inside this row, or every row is done
          ++row;  // this own row is done: the next one
          const uint32_t a = row == 1 ? p1 + adj1 : p2 + adj2;
          u = a + (uint32_t)q;
          uend = a + (row == 1 ? p2 - p1 : no - p2);
        }
        flush();
      }
    }
  }
}

// Visit the candidates of the 3x3 block of cells around cell K (rows bottom
// to top, cells left to right, sorted order inside a cell), dealt
// round-robin to a group of G lanes (lane l takes c = l, l + G, ...) with
// SCAN_UNROLL loads in flight. fn gets the candidate's pv and aux and its
// cell-shift code (row << 2) | column.
// The empty asm statement takes every loaded value (as an operand it may
// change), so the group's loads all complete there, together: otherwise
// the compiler defers the loads of the fields that fn reads only in support
// into fn's branches, and a lane waits for them one candidate at a time.
template <int G, class Fn>
__device__ __forceinline__ void for_candidates(const Dev& d, const InstParams& P, const Buf& sb, uint32_t K,
                                               int lane, Fn&& fn) {
  int cx, cy;
  cell_xy(P, K, cx, cy);
  const RowRange r0 = row_range(d, P, cx, cy, -1), r1 = row_range(d, P, cx, cy, 0),
                 r2 = row_range(d, P, cx, cy, 1);
  const uint32_t n0 = r0.re - r0.rs, n01 = n0 + (r1.re - r1.rs), n = n01 + (r2.re - r2.rs);
  for (uint32_t c0 = (uint32_t)lane; c0 < n; c0 += G * SCAN_UNROLL) {
    uint32_t code[SCAN_UNROLL];
    float4 pq[SCAN_UNROLL], aq[SCAN_UNROLL];
#pragma unroll
    for (int u = 0; u < SCAN_UNROLL; ++u) {
      const uint32_t c = min(c0 + G * u, n - 1);
      const uint32_t row = c < n0 ? 0u : (c < n01 ? 1u : 2u);
      const RowRange& r = row == 0 ? r0 : (row == 1 ? r1 : r2);
      const uint32_t j = r.rs + c - (row == 0 ? 0u : (row == 1 ? n0 : n01));
      code[u] = (row << 2) | dx_code(j, r);
      pq[u] = at32(sb.pv, j);
      aq[u] = at32(sb.aux, j);
    }
#pragma unroll
    for (int u = 0; u < SCAN_UNROLL; ++u)
      asm("" : "+v"(pq[u].x), "+v"(pq[u].y), "+v"(pq[u].z), "+v"(pq[u].w), "+v"(aq[u].x), "+v"(aq[u].y),
          "+v"(aq[u].z), "+v"(aq[u].w));
#pragma unroll
    for (int u = 0; u < SCAN_UNROLL; ++u)
      if (c0 + G * u < n) fn(pq[u], aq[u], code[u]);
  }
}
// r_a - r_j for a point at offset (ox, oy) of the centre cell and a candidate
// with shift code `code`
__device__ __forceinline__ void rel_pos(const InstParams& P, float ox, float oy, const float4& pj, uint32_t code,
                                        float& rx, float& ry) {
  rx = (ox - pj.x) - ((float)(int)(code & 3u) - 1.0f) * P.dc;
  ry = (oy - pj.y) - ((float)(int)(code >> 2) - 1.0f) * P.dc;
}

// Sum over a group of G consecutive lanes (xor butterfly: fixed order, the
// same bits on every lane of the group).
template <int G>
__device__ __forceinline__ float group_sum(float v) {
  for (int o = 1; o < G; o <<= 1) v += __shfl_xor(v, o);
  return v;
}
template <int G>
__device__ __forceinline__ double group_sum(double v) {
  for (int o = 1; o < G; o <<= 1) v += __shfl_xor(v, o);
  return v;
}

// Shepard sums over the fluid in support of an encoded point (cell K,
// offset o), one group of G lanes per point.
struct Shep {
  float W, p, rx, ry, vx, vy;
};
template <int G, bool CUB>
__device__ __forceinline__ Shep shepard(const Dev& d, const InstParams& P, const Buf& sb, uint32_t K, float ox,
                                        float oy, int lane) {
  Shep S = {0, 0, 0, 0, 0, 0};
  for_candidates<G>(d, P, sb, K, lane, [&](const float4& pj, const float4& aj, uint32_t code) __attribute__((always_inline)) {
    float rx, ry;  // r_g - r_j
    rel_pos(P, ox, oy, pj, code, rx, ry);
    const float r2 = rx * rx + ry * ry;
    if (!(aj.w > 0.0f) || !(r2 < P.four_h2)) return;  // fluid in support only
    float W, F;
    if constexpr (CUB) cubic_spline(P, r2, W, F);
    else wendland(P, r2, W, F);
    const float pj_ = aj.y * aj.x * aj.x;  // p = P rho^2
    S.W += W;
    S.p += pj_ * W;
    S.rx += aj.x * rx * W;
    S.ry += aj.x * ry * W;
    S.vx += pj.z * W;
    S.vy += pj.w * W;
  });
  S.W = group_sum<G>(S.W);
  S.p = group_sum<G>(S.p);
  S.rx = group_sum<G>(S.rx);
  S.ry = group_sum<G>(S.ry);
  S.vx = group_sum<G>(S.vx);
  S.vy = group_sum<G>(S.vy);
  return S;
}

}  // namespace

// ---------------------------------------------------------------------------
// Clock of one instance at the start of an evaluation (one thread):
//   EV_A     commit the previous step (t = t_next, step + 1), evaluate at t
//   EV_B     dt of the step from v_max (or the fixed table), start the next
//            v_max, record (t, dt); evaluate at t + dt/2
//   EV_EXPORT evaluate the newest state at t_next without advancing
// The disk kinematics at the evaluation time feed the ghost kernel.
template <int MODE>
__device__ void clock_commit(const Dev& d, int i) {
  const InstParams& P = d.prm[i];
  Clock& C = d.clk[i];
  double te;
  if (MODE == EV_A || MODE == EV_L) {
    C.t = C.t_next;
    C.step += 1;
    te = C.t;
    if (P.kin_mode == 2) {
      if (C.coupled) {
        C.xc = C.xd_next;
        C.vc = C.vd_next;
        C.ac = C.ac_next;
      } else if (C.t >= P.kin_t_ramp) {
        // the first step at or after the ramp starts from the prescribed state
        double x0, v0, a0;
        kinematics(P, C.t, x0, v0, a0);
        C.xc = x0;
        C.vc = v0;
        C.ac = a0;
        C.coupled = 1;
      }
    }
  } else if (MODE == EV_B) {
    const double dt = step_dt(d, P, C);
    C.dt = dt;
    C.vmax_used = (double)__uint_as_float(C.vmax_bits);
    C.vmax_bits = 0u;
    const long long row = (long long)i * WC_HIST_CAP + (C.step % WC_HIST_CAP);
    d.hist_t[row] = C.t;
    d.hist_dt[row] = dt;
    te = C.t + 0.5 * dt;
    if (!(P.kin_mode == 2 && C.coupled)) {  // a coupled disk's new state comes from k_disk
      double xn, vn, an;
      kinematics(P, C.t + dt, xn, vn, an);
      C.xd_next = xn;
      C.vd_next = vn;
    }
  } else {
    te = C.t_next;
  }
  double x, v, a;
  if (MODE == EV_EXPORT) disk_newest(P, C, x, v, a);
  else disk_at(P, C, te, x, v, a);
  C.t_eval = te;
  C.xd = x;
  C.vd = v;
  C.ad = a;
}

// A cell holds more slots than its bucket: flag the state (once).
__device__ __forceinline__ void flag_overflow(const Dev& d) {
  if (!(__hip_atomic_load(&d.clk[0].bad, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & 8u))
    atomicOr(&d.clk[0].bad, 8u);
}

// The bucket set one evaluation fills for the next sort: the cell buckets,
// and per sort tile (WC_SORT_TILE cells) the number of entries, so that the
// sort finds each tile's place without a scan across blocks.
struct Fill {
  uint32_t* bucket;
  uint32_t* tot;
};
__device__ __forceinline__ Fill fill_a(const Dev& d) { return Fill{d.bucket_a, d.tot_a}; }
__device__ __forceinline__ Fill fill_b(const Dev& d) { return Fill{d.bucket_b, d.tot_b}; }
#define WC_TILE_SHIFT 6   // log2 WC_SORT_TILE
static_assert(WC_SORT_TILE == 1 << WC_TILE_SHIFT, "tile shift");

// Slot s into the bucket of cell K for the next sort (bucket slot from the
// cell's fill counter); an overfull cell is flagged and the slot dropped
// (its tile still counts it, so every later slot keeps its place).
__device__ __forceinline__ void bucket_put(const Dev& d, const Fill& f, uint32_t K, uint32_t s) {
  const uint32_t b = atomicAdd(&d.count[K], 1u);
  if (b < WC_BUCKET) f.bucket[(size_t)K * WC_BUCKET + b] = s;
  else flag_overflow(d);
  atomicAdd(&f.tot[K >> WC_TILE_SHIFT], 1u);
}

// Runs of consecutive active lanes (mask A) with the same value v: whether
// this lane heads its run, the run's head lane h and length (on the head).
struct Run {
  bool head;
  int h;
  uint32_t len, rank;
};
__device__ __forceinline__ Run lane_run(unsigned long long A, bool act, uint32_t v) {
  const int lane = (int)(threadIdx.x & 63);
  // previous active lane (below this one) and its value
  const unsigned long long below = A & ((1ull << lane) - 1ull);
  const int prev = below ? 63 - __clzll((long long)below) : -1;
  const uint32_t vprev = __shfl(v, prev < 0 ? lane : prev);
  Run r;
  r.head = act && (prev < 0 || vprev != v);
  const unsigned long long H = __ballot(r.head);
  // this lane's run head and the next head above it
  const unsigned long long upto = (lane == 63) ? ~0ull : ((1ull << (lane + 1)) - 1ull);
  const unsigned long long hb = H & upto;
  r.h = hb ? 63 - __clzll((long long)hb) : 0;
  const unsigned long long above = H & ~upto;
  const int nh = above ? __ffsll((long long)above) - 1 : 64;
  const unsigned long long from_h = ~((1ull << r.h) - 1ull);
  const unsigned long long to_nh = nh == 64 ? ~0ull : ((1ull << nh) - 1ull);
  r.len = (uint32_t)__popcll(A & from_h & to_nh);
  r.rank = (uint32_t)__popcll(A & from_h & ((1ull << lane) - 1ull));
  return r;
}

// bucket_put for the lanes with `act` set, one atomic per run: consecutive
// active lanes (slots in sorted order, mostly keeping their cell) with the
// same key share one fill-counter update and take consecutive bucket slots;
// the tile totals take one (non-returning) atomic per run of their own.
__device__ __forceinline__ void bucket_put_wave(const Dev& d, const Fill& f, bool act, uint32_t K, uint32_t s) {
  const unsigned long long A = __ballot(act);
  if (A == 0ull) return;
  const Run rk = lane_run(A, act, K);
  uint32_t b0 = 0;
  if (rk.head) b0 = atomicAdd(&d.count[K], rk.len);
  const Run rt = lane_run(A, act, K >> WC_TILE_SHIFT);
  if (rt.head) atomicAdd(&f.tot[K >> WC_TILE_SHIFT], rt.len);
  b0 = __shfl(b0, rk.h);
  if (!act) return;
  const uint32_t b = b0 + rk.rank;
  if (b < WC_BUCKET) f.bucket[(size_t)K * WC_BUCKET + b] = s;
  else flag_overflow(d);
}

// Wall ghost g (static position) into its fixed place at the front of its bucket.
// (Wall ghosts are counted in the static per-cell and per-tile totals the
// counters are re-armed with.)
__device__ __forceinline__ void bucket_put_wall(const Dev& d, const InstParams& P, const Fill& f, uint32_t K,
                                                int g, uint32_t s) {
  f.bucket[(size_t)K * WC_BUCKET + d.wrank[P.gmap0 + g]] = s;
}

// Disk-ring ghost k of instance inst for a disk centre at x = xc:
// r_k = (xc, y0) + R (cos 2 pi k / nd, sin 2 pi k / nd), encoded, and put
// into its bucket for the next sort.
__device__ __forceinline__ void place_ring(const Dev& d, const InstParams& P, int inst, int k, double xc,
                                           const Buf& out, int s, const Fill& bucket) {
  const double2 cs = d.ring_cs[inst * WC_MAX_RING + k];
  const double x = xc + P.R * cs.x, y = P.disk_y0 + P.R * cs.y;
  int cx, cy;
  float ox, oy;
  encode_axis(x, P.x_lo, P.dcd, P.inv_dcd, P.dc, P.ncx, cx, ox);
  encode_axis(y, P.y_lo, P.dcd, P.inv_dcd, P.dc, P.ncy, cy, oy);
  const uint32_t key = (uint32_t)(P.cell_off + cy * P.ncx + cx);
  out.cell[s] = key;
  out.pv[s] = make_float4(ox, oy, 0.0f, 0.0f);
  bucket_put(d, bucket, key, (uint32_t)s);
}

// ---------------------------------------------------------------------------
// The cell-list build of one evaluation in one launch: a stable counting
// sort of the slots by cell key. The previous evaluation left every slot in
// the bucket of its new cell (bucket order arbitrary, from atomics), and
// counted the entries per cell and per tile of WC_SORT_TILE cells. Block 0
// advances the clocks (a chain of dependent FP64 loads and stores that no
// tile waits for); block b > 0 owns the cells of tile b - 1, [(b-1) T, b T)
// (T = WC_SORT_TILE). Its first wave turns the
// cells' counts into local offsets and finds the tile's first sorted slot as
// the sum of the totals of the tiles before it (a few loads per lane, no
// waiting on other blocks) -> start[]. Meanwhile the other waves, four lanes per cell,
// copy each bucket into LDS, fetch the state of their entries, and rank each
// entry by old slot within its bucket (rank = number of smaller entries: the
// sort is stable with respect to the current order). After one block
// barrier every entry is stored at its sorted place with the per-particle
// EOS; ghost slots and perm[new] = old are recorded. Each tile re-arms its
// tile's total of the other bucket set with the static wall-ghost entries,
// for the fills of the evaluation that follows.
#define SORT_CELL_WAVES (WC_SORT_TILE / 16)     // four lanes per cell
#define SORT_BLOCK (64 * (1 + SORT_CELL_WAVES))  // plus the offsets wave
#define SORT_SPEC 3  // bucket entries per lane fetched with the counts
#ifndef SORT_PRE
#define SORT_PRE 8  // tile totals per lane in flight at once in the tile prefix
#endif
#define SORT_FOLD 16  // per-block v_max entries per lane in flight in the fold

// State of one particle at its old slot e, as loaded (before the EOS).
struct Loaded {
  uint32_t cell, id;
  float4 pv;
  float rho, e;  // e: scheme 1 internal energy
  int inst;  // -1: corrupted bucket entry
};
// One particle moved by the sort: its state with the per-particle EOS
// (fluid) or ghost mass.
struct Gathered {
  uint32_t cell, id;
  float4 pv, aux;
  float e;
  int inst, ghost;  // ghost: -1 for fluid, else the ghost index g of its instance
};
// (branch-free: an entry outside the slot range reads slot 0 and is marked)
template <bool BATCH>
__device__ __forceinline__ Loaded sort_load(const Dev& d, const Buf& pre, uint32_t e) {
  Loaded v;
  const bool ok = e < (uint32_t)d.n_slots;  // else a corrupted bucket: flagged when stored
  const uint32_t x = ok ? e : 0u;
  v.inst = inst_at<BATCH>(pre, (int)x);
  v.cell = pre.cell[x];
  v.id = pre.id[x];
  v.pv = pre.pv[x];
  v.rho = pre.aux[x].x;
  v.e = pre.e ? pre.e[x] : 0.0f;
  if (!ok) v.inst = -1;
  return v;
}
template <bool MG>
__device__ __forceinline__ Gathered sort_finish(const Dev& d, const Loaded& l) {
  Gathered v;
  v.inst = l.inst;
  if (l.inst < 0) return v;
  const InstParams& P = d.prm[l.inst];
  v.cell = l.cell;
  v.id = l.id;
  v.pv = l.pv;
  v.e = l.e;
  const int local = (int)l.id - P.id0;
  if (local < P.nf) {
    float Pq = 0.0f, c = 0.0f;
    // (scheme 1: the density pass that follows sums the density and applies the EOS)
    if (P.scheme == 0) fluid_eos<MG>(P, l.rho, Pq, c);
    float m = P.m_fluid;
    if (P.axisym) {
      // the ring's planar mass M / (2 pi r), r held >= dx/2
      int cx, cy;
      cell_xy(P, l.cell, cx, cy);
      const double r = P.y_lo + (double)cy * P.dcd + (double)l.pv.y;
      m = (float)(d.mring[l.id] / fmax(r, P.r_mind));
    }
    v.aux = make_float4(l.rho, Pq, c, m);
    v.ghost = -1;
  } else {
    v.ghost = local - P.nf;
    v.aux = make_float4(l.rho, 0.0f, 0.0f, v.ghost < P.nw ? -P.m_wall : -P.m_disk);
  }
  return v;
}
template <bool BATCH>
__device__ __forceinline__ void sort_store(const Dev& d, const Buf& out, uint32_t e, uint32_t dst,
                                           const Gathered& v) {
  if (v.inst < 0 || dst >= (uint32_t)d.n_slots) {
    atomicOr(&d.clk[0].bad, 4u);
    return;
  }
  if (v.ghost >= 0) {
    const int gi = d.prm[v.inst].gmap0 + v.ghost;
    d.gslot[gi] = dst;
    d.gcell[gi] = v.cell;
    d.gpos[gi] = make_float2(v.pv.x, v.pv.y);
  }
  out.cell[dst] = v.cell;
  out.id[dst] = v.id;
  out.pv[dst] = v.pv;
  out.aux[dst] = v.aux;
  if constexpr (BATCH) out.inst[dst] = (uint16_t)v.inst;
  if (out.e) out.e[dst] = v.e;
  d.perm[dst] = e;
}

template <int MODE, bool BATCH, bool MG>
__global__ __launch_bounds__(SORT_BLOCK) void k_sort(Dev d, Buf pre, Buf out) {
  constexpr int T = WC_SORT_TILE;
  __shared__ uint32_t s_off[T + 1];  // exclusive offsets of the tile's cells, total at [T]
  __shared__ uint32_t s_base;        // sorted slots before this tile
  __shared__ uint32_t s_raw[T * WC_BUCKET];
  const int t = threadIdx.x;
  if (blockIdx.x == 0) {
    if (t < 64) {
      for (int i = t; i < d.n_inst; i += 64) clock_commit<MODE>(d, i);
    } else if ((MODE == EV_A || MODE == EV_L) && !BATCH) {
      // meanwhile, single instance: the other waves fold the previous
      // corrector's per-block fluid maxima into the clock (SORT_FOLD loads
      // per lane in flight at once; a clamped index reads an entry again,
      // which leaves the maximum as it is), one atomic per wave; the commit
      // of a first evaluation does not read v_max
      constexpr int FL = SORT_BLOCK - 64;
      float vp = 0.0f;
      for (int i0 = t - 64; i0 < d.n_vpart; i0 += FL * SORT_FOLD) {
        float v[SORT_FOLD];
#pragma unroll
        for (int k = 0; k < SORT_FOLD; ++k) v[k] = d.vmax_part[min(i0 + FL * k, d.n_vpart - 1)];
#pragma unroll
        for (int k = 0; k < SORT_FOLD; ++k) vp = fmaxf(vp, v[k]);
      }
      const float w = wave_max(vp);
      if ((t & 63) == 0 && w > 0.0f) atomicMax(&d.clk[0].vmax_bits, __float_as_uint(w));
    }
    return;
  }
  const int tile = blockIdx.x - 1;
  // the bucket set this sort reads: b for the corrector, the step's set for
  // a leapfrog step, else a
  const bool set_b = MODE == EV_B || (MODE == EV_L && d.lf_set != 0);
  const uint32_t* bucket = set_b ? d.bucket_b : d.bucket_a;
  // cell lanes: lane sub of cell c owns the entries sub + 4 u of its bucket
  const int ct = t - 64, c = ct >> 2, sub = ct & 3;
  uint32_t n = 0u, e[SORT_SPEC], r[SORT_SPEC];
  Loaded lv[SORT_SPEC];
  Gathered gv[SORT_SPEC];
  if (t < 64) {
    // the tile's local offsets, and the sorted slots before the tile: the
    // entry totals of the tiles before it (filled with the buckets)
    const int K = tile * T + t;
    const uint32_t* tot = set_b ? d.tot_b : d.tot_a;
    const uint32_t cnt_raw = d.count[min(K, d.n_cells - 1)];  // in flight during the prefix
    // SORT_PRE loads in flight per lane and round (an index past the
    // preceding tiles reads the last of them and adds nothing), so the last
    // tiles wait for one round of latency, not one per 64 tiles
    uint32_t excl = 0u;
    for (int u0 = t; u0 < tile; u0 += 64 * SORT_PRE) {
      uint32_t v[SORT_PRE];
#pragma unroll
      for (int k = 0; k < SORT_PRE; ++k) v[k] = tot[min(u0 + 64 * k, tile - 1)];
#pragma unroll
      for (int k = 0; k < SORT_PRE; ++k) excl += u0 + 64 * k < tile ? v[k] : 0u;
    }
    const uint32_t cnt = K < d.n_cells ? min(cnt_raw, (uint32_t)WC_BUCKET) : 0u;  // overflow was flagged
    uint32_t incl = cnt;
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t u = __shfl_up(incl, o);
      if (t >= o) incl += u;
    }
    const uint32_t total = __shfl(incl, 63);
    s_off[t] = incl - cnt;
    if (t == 63) s_off[T] = total;
    for (int o = 32; o > 0; o >>= 1) excl += __shfl_xor(excl, o);
    // re-arm the other bucket set's total of this tile
    if (t == 0) (set_b ? d.tot_a : d.tot_b)[tile] = d.wall_tot[tile];
    if (t == 0) s_base = excl;
    if (K < d.n_cells) d.start[K] = excl + (incl - cnt);
    if (K == d.n_cells - 1) d.start[d.n_cells] = excl + incl;
  } else {
    const int K = tile * T + c;
    if (K < d.n_cells) {
      n = min(d.count[K], (uint32_t)WC_BUCKET);
#pragma unroll
      for (int u = 0; u < SORT_SPEC; ++u) e[u] = bucket[(size_t)K * WC_BUCKET + sub + 4 * u];
    } else {
#pragma unroll
      for (int u = 0; u < SORT_SPEC; ++u) e[u] = 0u;
    }
    uint32_t* raw = s_raw + c * WC_BUCKET;
#pragma unroll
    for (int u = 0; u < SORT_SPEC; ++u)
      if ((uint32_t)(sub + 4 * u) < n) raw[sub + 4 * u] = e[u];
    // the state of the lane's entries is in flight during the ranking and
    // the offsets (issued without branches; entries past the count load
    // slot 0 and are not used)
#pragma unroll
    for (int u = 0; u < SORT_SPEC; ++u) lv[u] = sort_load<BATCH>(d, pre, (uint32_t)(sub + 4 * u) < n ? e[u] : 0u);
    for (uint32_t i = sub + 4 * SORT_SPEC; i < n; i += 4) raw[i] = bucket[(size_t)K * WC_BUCKET + i];
    wave_sync();  // the buckets of this wave's cells are in LDS
    // rank of each entry in its bucket; the first 16 places without branches
#pragma unroll
    for (int u = 0; u < SORT_SPEC; ++u) r[u] = 0u;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const uint32_t x = raw[k];
#pragma unroll
      for (int u = 0; u < SORT_SPEC; ++u) r[u] += (((uint32_t)k < n) & (x < e[u])) ? 1u : 0u;
    }
    for (uint32_t k = 16; k < n; ++k) {
      const uint32_t x = raw[k];
#pragma unroll
      for (int u = 0; u < SORT_SPEC; ++u) r[u] += x < e[u] ? 1u : 0u;
    }
#pragma unroll
    for (int u = 0; u < SORT_SPEC; ++u) gv[u] = sort_finish<MG>(d, lv[u]);  // EOS while the offsets are found
  }
  __syncthreads();  // offsets and the tile's base
  if (t < 64) {
    const int K = tile * T + t;
    if (K < d.n_cells) d.count[K] = d.wallcount[K];  // re-arm for the next sort (every count was read)
    // a cell that took more entries than its bucket (flagged when filled)
    // leaves a gap in the tile's slot range, and the particles it dropped
    // leave the slots past the last tile unfilled from then on: both are
    // filled with inert entries (no particle id, zero mass, the tile's last
    // cell, old slot 0) so that every sorted slot holds a valid cell key and
    // a finite state that no later kernel moves or counts
    const uint32_t* tot = set_b ? d.tot_b : d.tot_a;
    const uint32_t stored = s_off[T];
    const uint32_t end = tile == (int)gridDim.x - 2 ? (uint32_t)d.n_slots - s_base : tot[tile];
    const uint32_t kin = (uint32_t)min(tile * T + T - 1, d.n_cells - 1);
    for (uint32_t g = stored + (uint32_t)t; g < end; g += 64) {
      const uint32_t dst = s_base + g;
      if (dst >= (uint32_t)d.n_slots) break;
      out.cell[dst] = kin;
      out.id[dst] = WC_NO_ID;
      out.pv[dst] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      out.aux[dst] = make_float4(1.0f, 0.0f, 0.0f, 0.0f);
      if constexpr (BATCH) out.inst[dst] = 0;
      if (out.e) out.e[dst] = 0.0f;
      d.perm[dst] = 0u;
    }
    return;
  }
  const uint32_t base = s_base + s_off[c];
#pragma unroll
  for (int u = 0; u < SORT_SPEC; ++u)
    if ((uint32_t)(sub + 4 * u) < n) sort_store<BATCH>(d, out, e[u], base + r[u], gv[u]);
  const uint32_t* raw = s_raw + c * WC_BUCKET;
  for (uint32_t i = sub + 4 * SORT_SPEC; i < n; i += 4) {
    const uint32_t ei = raw[i];
    uint32_t ri = 0u;
    for (uint32_t k = 0; k < n; ++k) ri += raw[k] < ei ? 1u : 0u;
    sort_store<BATCH>(d, out, ei, base + ri, sort_finish<MG>(d, sort_load<BATCH>(d, pre, ei)));
  }
}

// Adami ghost state (walls and ring), probes, ghost v_max and ring work.
// WC_GHOST_LANES lanes per ghost or probe share its 3x3 candidates. Block
// table entry: (instance, first item, item count, kind); kind 0 wall ghosts,
// 1 ring ghosts, 2 probes.
#define GL WC_GHOST_LANES
template <int MODE, bool BATCH, bool CUB>
__global__ __launch_bounds__(WC_GHOST_BLOCK) void k_ghost(Dev d, Buf sb) {
  // the table entry in one load, and (single instance) the offset of the
  // instance's ghost arrays with it: left to itself the compiler loads each
  // field where it is first used, one after the other
  int4 blk = d.gblk[blockIdx.x];
  int gm = BATCH ? 0 : d.prm[0].gmap0;
  const uint32_t *gslot = d.gslot, *gcell = d.gcell;
  const float2* gpos = d.gpos;
  asm("" : "+s"(blk.x), "+s"(blk.y), "+s"(blk.z), "+s"(blk.w), "+s"(gm), "+s"(gslot), "+s"(gcell), "+s"(gpos));
  const int inst = BATCH ? blk.x : 0, kind = blk.w;
  const InstParams& P = d.prm[inst];
  if constexpr (BATCH) gm = P.gmap0;
  Clock& C = d.clk[inst];
  const int t = threadIdx.x, item = t / GL, lane = t % GL;
  const bool act = item < blk.z;
  // first evaluation: the stored v_max (the fluid part is already in) read
  // now, so that its latency is hidden; a wave whose ghost maximum is not
  // above it skips the atomic
  constexpr bool FIRST = MODE == EV_A || MODE == EV_L;  // the step's first (or only) evaluation
  const uint32_t vcheck = FIRST && kind != 2 ? __atomic_load_n(&C.vmax_bits, __ATOMIC_RELAXED) : 0u;
  if (kind == 2) {
    // probes: Shepard average of the fluid pressure at fixed wall points
    if (FIRST && act) {
      const int k = blk.y + item;
      const Shep S = shepard<GL, CUB>(d, P, sb, P.probe_cell[k], P.probe_ox[k], P.probe_oy[k], lane);
      if (lane == 0) {
        const long long row = (long long)inst * WC_HIST_CAP + (C.step % WC_HIST_CAP);
        d.hist_p[row * WC_MAX_PROBES + k] = S.W > 0.0f ? S.p / S.W : 0.0f;
      }
    }
    return;
  }
  const bool disk = kind == 1;
  float vmag = 0.0f;
  if (act) {
    const int g = blk.y + item;
    const uint32_t s = gslot[gm + g];
    const uint32_t K = gcell[gm + g];
    const float2 pg = gpos[gm + g];
    // axisymmetric form: a wall ghost below the axis mirrors the fluid (slip)
    // and is off (zero mass, at rest) inside the sphere
    bool axis = false, off = false;
    if (P.axisym && !disk) {
      int gcx, gcy;
      cell_xy(P, K, gcx, gcy);
      const double yg = P.y_lo + (double)gcy * P.dcd + (double)pg.y;
      axis = yg < 0.0;
      if (axis && P.nd > 0) {
        const double xg = P.x_lo + (double)gcx * P.dcd + (double)pg.x;
        const double ux = xg - C.xd, uy = yg - P.disk_y0;
        off = ux * ux + uy * uy < P.R * P.R;  // the same on every lane of the item
      }
    }
    if (off) {
      if (lane == 0) {
        sb.pv[s] = make_float4(pg.x, pg.y, 0.0f, 0.0f);
        sb.aux[s] = make_float4(P.rho0, 0.0f, P.c0, -0.0f);
      }
    } else {
      const Shep S = shepard<GL, CUB>(d, P, sb, K, pg.x, pg.y, lane);
      const float vwx = disk ? (float)C.vd : 0.0f;
      const float awx = disk ? (float)C.ad : 0.0f;
      float p, vgx, vgy;
      if (S.W > 0.0f) {
        const float inv = 1.0f / S.W;
        // body-force term (g - a_w) . sum rho_j (r_g - r_j) W
        p = (S.p + (0.0f - awx) * S.rx + P.gy * S.ry) * inv;
        vgx = axis ? S.vx * inv : 2.0f * vwx - S.vx * inv;  // axis: the axial velocity is kept
        vgy = -S.vy * inv;
      } else {
        p = 0.0f;
        vgx = vwx;
        vgy = 0.0f;
      }
      p = fmaxf(p, P.p_cav);
      float rg, cg;
      if (P.eos_type == 1) {
        // Mie-Grueneisen inverse: tension line, or the root in [0, 1/b) of
        // s (1 - b mu)^2 = mu (1 + k1 mu), s = p / K; capped at mu_max
        const float sp = p / P.mg_K;
        float mu = sp;
        if (P.ghost_rho_mode != 0 && sp > 0.0f)
          mu = fminf(2.0f * sp / ((1.0f + 2.0f * P.mg_b * sp) + sqrtf(1.0f + 4.0f * sp * (P.mg_b + P.mg_k1))),
                     P.mg_mu_max);
        rg = P.rho0 * (1.0f + mu);
        float pu;
        mg_eos(P, mu, pu, cg);
      } else {
        if (P.ghost_rho_mode == 0) rg = P.rho0 * (1.0f + p * P.inv_rho0c02);
        else rg = P.rho0 * expf(P.inv_gamma * log1pf(p / P.B));
        const float xg = (rg - P.rho0) / P.rho0, yg = 1.0f + xg;
        cg = P.gamma == 7.0f ? P.c0 * (yg * yg * yg) : P.c0 * expf(P.c_exp * log1pf(xg));
      }
      const float Pg = p / (rg * rg);
      const float m = disk ? P.m_disk : P.m_wall;
      if (lane == 0) {
        sb.pv[s] = make_float4(pg.x, pg.y, vgx, vgy);
        sb.aux[s] = make_float4(rg, Pg, cg, -m);
        vmag = fast_sqrt(vgx * vgx + vgy * vgy);
      }
      if ((MODE == EV_B || MODE == EV_L) && disk) {
        // x force of this ring ghost on its fluid neighbours (pressure + AV)
        float fx = 0.0f;
        int rcx, rcy;
        cell_xy(P, K, rcx, rcy);
        const float yg = (float)(P.y_lo + (double)rcy * P.dcd) + pg.y;  // the ghost's radius (axisymmetric)
        for_candidates<GL>(d, P, sb, K, lane, [&](const float4& pj, const float4& aj, uint32_t code) __attribute__((always_inline)) {
          if (!(aj.w > 0.0f)) return;
          float rx, ry;
          rel_pos(P, pg.x, pg.y, pj, code, rx, ry);
          rx = -rx;  // r_i - r_g
          ry = -ry;
          const float r2 = rx * rx + ry * ry;
          if (!(r2 < P.four_h2)) return;
          float W, F;
          if constexpr (CUB) cubic_spline(P, r2, W, F);
          else wendland(P, r2, W, F);
          const float vr = (pj.z - vgx) * rx + (pj.w - vgy) * ry;
          const float rsum = aj.x + rg, den = r2 + P.eta2h2;
          const float inv = fast_rcp(den * rsum);
          const float piav =
              vr < 0.0f ? -P.alpha * (aj.z + cg) * P.h * vr * inv + P.beta2h2 * vr * vr * inv * (rsum * inv) : 0.0f;
          // (axisymmetric: the fluid particle's ring mass 2 pi m r in place of m)
          const float mi = P.axisym ? aj.w * (6.283185307f * fmaxf(yg + ry, P.r_min)) : aj.w;
          fx -= mi * m * (aj.y + Pg + piav) * F * rx;
        });
        const double f = group_sum<GL>((double)fx);
        if (lane == 0) d.wb_part[inst * WC_MAX_RING + (g - P.nw)] = f;
      }
    }
  }
  if (FIRST) {
    // the items of a block belong to one instance
    const float w = wave_max(vmag);
    if ((t & 63) == 0 && w > 0.0f && __float_as_uint(w) > vcheck) atomicMax(&C.vmax_bits, __float_as_uint(w));
  }
}
#undef GL

// Pair sums + predictor (eval A) / corrector (eval B) for every fluid slot;
// ghost slots are carried into the output buffer. EV_EXPORT writes the rates.
// A block serves PAIR_SLOTS consecutive slots: first every wave sums the pair
// law with four lanes per slot, then the first wave finishes the slots with
// one lane each (time integration, enforcement, bucket entries), so the
// per-slot FP64 work runs on full waves.
// r^(gamma - 1) in FP64: repeated products for an integer gamma (the Tait
// gamma = 7 gives r^6), pow otherwise.
__device__ __forceinline__ double pow_gm1(double r, double g) {
  const double e = g - 1.0;
  if (e == floor(e) && e >= 0.0 && e <= 16.0) {
    double p = 1.0, b = r;
    for (int k = (int)e; k > 0; k >>= 1) {
      if (k & 1) p *= b;
      b *= b;
    }
    return p;
  }
  return pow(r, e);
}

// Specific elastic energy of the Tait law with the cutoff branch below
// rho_c (the diagnostics' closed form), FP64.
__device__ __forceinline__ double tait_e_el(const InstParams& P, double r) {
  const double rg1 = pow_gm1(r, P.gammad);
  return r >= P.diag_rc ? P.diag_k1 * (rg1 - P.diag_r0g1) + P.Bd * (1.0 / r - 1.0 / P.rho0d)
                        : P.diag_erc + P.p_cavd * (1.0 / P.diag_rc - 1.0 / r);
}

// Specific elastic energy of the Mie-Grueneisen law at zero internal energy
// (int p / rho^2 drho from rho0), FP64. Per unit mu the integrand is
// p(mu) / (rho0 (1 + mu)^2): 8-point Gauss-Legendre on the smooth piece from
// 0 to mu clamped to [mu_cav, mu_max], the constant-pressure pieces beyond
// the cutoff and the cap in closed form.
__device__ __forceinline__ double mg_e_el(const InstParams& P, double r) {
  constexpr double xg[4] = {0.18343464249564978, 0.52553240991632899, 0.79666647741362673, 0.96028985649753618};
  constexpr double wg[4] = {0.36268378337836177, 0.31370664587788705, 0.22238103445337434, 0.10122853629037669};
  const double mu = r / P.rho0d - 1.0;
  const double m = fmin(fmax(mu, P.mg_mu_cavd), P.mg_mu_maxd);
  double sum = 0.0;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const double u = 0.5 * m * (1.0 + ((k & 1) ? -xg[k >> 1] : xg[k >> 1]));
    const double den = 1.0 - P.mg_bd * u;
    const double p = m >= 0.0 ? P.mg_Kd * u * (1.0 + P.mg_k1d * u) / (den * den) : P.mg_Kd * u;
    sum += wg[k >> 1] * p / ((1.0 + u) * (1.0 + u));
  }
  double e = 0.5 * m * sum / P.rho0d;
  if (mu > m) e += P.mg_p_capd / P.rho0d * (1.0 / (1.0 + m) - 1.0 / (1.0 + mu));
  else if (mu < m) e += P.p_cavd / P.rho0d * (1.0 / (1.0 + m) - 1.0 / (1.0 + mu));
  return e;
}
__device__ __forceinline__ double eos_e_el(const InstParams& P, double r) {
  return P.eos_type == 1 ? mg_e_el(P, r) : tait_e_el(P, r);
}

// Blocks per compute unit the register budget of the single-instance pair
// pass is held to: seven (seven waves per SIMD, at most 72 VGPRs), which it
// meets without spills; left to itself the compiler took 79 VGPRs (six waves
// per SIMD) and the pass ran 6 % slower (C2). The batched, audit, export
// and cubic-kernel variants keep the compiler's budget (they would spill).
#ifndef PAIR_MINW
#define PAIR_MINW 7
#endif
template <int MODE, bool BATCH, bool AUD, int VAR>
__global__ __launch_bounds__(PAIR_BLOCK, (BATCH || AUD || MODE == EV_EXPORT || (VAR & 2)) ? 1 : PAIR_MINW)
void k_pair(Dev d, Buf sb, Buf base, Buf out) {
  __shared__ float4 uni[PAIR_BLOCK / 64][UCAP];
  __shared__ uint8_t lst[LCAP * PAIR_BLOCK];
  // hand-over of each slot from the first phase to the second
  __shared__ float sacc[5][PAIR_SLOTS];
  __shared__ float4 h_pv[PAIR_SLOTS];
  __shared__ uint32_t h_K[PAIR_SLOTS], h_id[PAIR_SLOTS], h_eb[PAIR_SLOTS];
  __shared__ float h_rho[PAIR_SLOTS], h_m[PAIR_SLOTS];
  __shared__ int h_inst[PAIR_SLOTS];
  __shared__ float h_aud[AUD ? 4 : 1][PAIR_SLOTS];
  // a single instance's constants and clock, copied for the second phase:
  // the compiler cannot move global loads above the phase's global stores,
  // and waited for each field in turn; from LDS it loads them together
  // (no block writes a clock field that a second phase reads)
  __shared__ InstParams sP;
  __shared__ Clock sC;
  if constexpr (!BATCH) {
    constexpr int NP = (int)(sizeof(InstParams) / 4), NC = (int)(sizeof(Clock) / 4);
    static_assert(sizeof(InstParams) % 4 == 0 && sizeof(Clock) % 4 == 0 && NP + NC <= PAIR_BLOCK, "copy");
    const int t = (int)threadIdx.x;
    if (t < NP) reinterpret_cast<uint32_t*>(&sP)[t] = reinterpret_cast<const uint32_t*>(d.prm)[t];
    else if (t < NP + NC) reinterpret_cast<uint32_t*>(&sC)[t - NP] = reinterpret_cast<const uint32_t*>(d.clk)[t - NP];
  }
  // blocks map to XCDs in contiguous slot ranges
  const int s0 = xcd_block(blockIdx.x, gridDim.x) * PAIR_SLOTS;
  {
    const int q = (int)(threadIdx.x % PAIR_G);
    const int s = s0 + (int)(threadIdx.x / PAIR_G);
    const bool inr = s < d.n_slots;
    const int inst = inr ? inst_at<BATCH>(sb, s) : 0;
    uint32_t K = 0;
    float4 pi = make_float4(0, 0, 0, 0), ai = make_float4(0, 0, 0, 0);
    if (inr) {
      K = sb.cell[s];
      pi = sb.pv[s];
      ai = sb.aux[s];
    }
    const bool fluid = inr && ai.w > 0.0f;
    // fetched now, used after the pair sums: the particle id and (eval B)
    // the slot of its state n in the step's first sorted state
    uint32_t id = 0u, eb = 0u;
    if (q == 0 && inr) {
      id = sb.id[s];
      if (MODE == EV_B && fluid) eb = d.perm[s];
    }
    PairAcc acc = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
    AudAcc aud = {0.0f, 0.0f, 0.0f, 0.0f};
    if (MODE == EV_EXPORT && d.nb_ids != nullptr)
      pair_sums_wave<BATCH, AUD, VAR, true>(d, sb, s, inst, K, fluid, pi, ai, q, uni[threadIdx.x >> 6],
                                            lst + threadIdx.x, acc, aud);
    else
      pair_sums_wave<BATCH, AUD, VAR>(d, sb, s, inst, K, fluid, pi, ai, q, uni[threadIdx.x >> 6],
                                      lst + threadIdx.x, acc, aud);
    // fixed-order combination of the slot's lane partial sums
    acc.D = slot_sum(acc.D);
    acc.ax = slot_sum(acc.ax);
    acc.ay = slot_sum(acc.ay);
    acc.Vx = slot_sum(acc.Vx);
    acc.Vy = slot_sum(acc.Vy);
    if (q == 0) {
      const int k = (int)(threadIdx.x / PAIR_G);
      sacc[0][k] = acc.D;
      sacc[1][k] = acc.ax;
      sacc[2][k] = acc.ay;
      sacc[3][k] = acc.Vx;
      sacc[4][k] = acc.Vy;
      h_pv[k] = pi;
      h_K[k] = K;
      h_rho[k] = ai.x;
      h_m[k] = inr ? ai.w : 0.0f;
      h_inst[k] = inst;
      h_id[k] = id;
      h_eb[k] = eb;
    }
    if constexpr (AUD) {
      aud.av = slot_sum(aud.av);
      aud.visc = slot_sum(aud.visc);
      aud.del = slot_sum(aud.del);
      aud.ghost = slot_sum(aud.ghost);
      if (q == 0) {
        const int k = (int)(threadIdx.x / PAIR_G);
        h_aud[0][k] = aud.av;
        h_aud[1][k] = aud.visc;
        h_aud[2][k] = ai.y * aud.del;  // elastic energy rate P_i drho_i of the delta term
        h_aud[3][k] = aud.ghost;
      }
    }
  }
  __syncthreads();
  if (threadIdx.x >= PAIR_SLOTS) return;
  const int s = s0 + (int)threadIdx.x;
  const bool inr = s < d.n_slots;
  const int inst = BATCH ? h_inst[threadIdx.x] : 0;
  const InstParams& P = *(BATCH ? &d.prm[inst] : &sP);
  Clock* clk = d.clk;
  const Clock& C = *(BATCH ? &clk[inst] : &sC);
  const uint32_t K = h_K[threadIdx.x];
  const float4 pi = h_pv[threadIdx.x];
  const float rho_i = h_rho[threadIdx.x];
  const uint32_t id_i = h_id[threadIdx.x];
  const bool fluid = inr && h_m[threadIdx.x] > 0.0f;
  const uint32_t eb = h_eb[threadIdx.x];
  const int gid = (int)id_i - P.id0 - P.nf;  // ghost index (an inert entry has none)
  // the bucket set this pass fills for the next sort
  const Fill next_fill = (MODE == EV_A || (MODE == EV_L && d.lf_set == 0)) ? fill_b(d) : fill_a(d);
  if (MODE != EV_EXPORT && inr && !fluid && gid >= 0 && gid < P.nw + P.nd) {
    // ghosts: wall ghosts are carried, the disk ring is placed at the time of
    // the next evaluation (t + dt/2 after eval A, t + dt after eval B or a
    // leapfrog step)
    const uint32_t id = id_i;
    const int ring = (int)id - P.id0 - P.nf - P.nw;
    out.id[s] = id;
    out.aux[s] = make_float4(rho_i, 0.0f, 0.0f, 0.0f);
    if constexpr (BATCH) out.inst[s] = (uint16_t)inst;
    if (out.e) out.e[s] = 0.0f;
    const Fill bucket = next_fill;
    if (ring >= 0) {
      double xc = C.xd_next;
      if (MODE == EV_A) {  // disk at t + dt/2
        double vc, ac;
        disk_at(P, C, C.t + 0.5 * step_dt(d, P, C), xc, vc, ac);
      }
      place_ring(d, P, inst, ring, xc, out, s, bucket);
    } else {
      out.cell[s] = K;
      out.pv[s] = pi;
      bucket_put_wall(d, P, bucket, K, (int)id - P.id0 - P.nf, (uint32_t)s);
    }
  }
  PairAcc acc;
  acc.D = sacc[0][threadIdx.x];
  acc.ax = sacc[1][threadIdx.x];
  acc.ay = sacc[2][threadIdx.x];
  acc.Vx = sacc[3][threadIdx.x];
  acc.Vy = sacc[4][threadIdx.x];
  const bool lead = fluid;
  if (P.axisym && lead) {
    // axisymmetric form: the hoop part of the divergence, -rho v_r / r (r >= dx/2)
    int cx, cy;
    cell_xy(P, K, cx, cy);
    const float r = fmaxf((float)(P.y_lo + (double)cy * P.dcd) + pi.y, P.r_min);
    acc.D -= rho_i * pi.w / r;
  }
  if (MODE == EV_EXPORT) {
    if (lead) {
      d.xr[s] = acc.D;
      d.xr[d.n_slots + s] = acc.ax;
      d.xr[2 * d.n_slots + s] = acc.ay + P.gy;
      d.xr[3 * d.n_slots + s] = pi.z + acc.Vx;
      d.xr[4 * d.n_slots + s] = pi.w + acc.Vy;
    }
    return;
  }
  bool clamp_hit = false, enf_hit = false;
  double e_enf = 0.0, e_clamp = 0.0;  // audit: energy of the enforcement and clamp
  float vnew = 0.0f;
  uint32_t newkey = 0u;
  if (lead) {
    const double dt = MODE == EV_A ? step_dt(d, P, C) : C.dt;
    const float hdt = (float)(MODE == EV_A ? 0.5 * dt : dt);
    uint32_t Kb;
    float4 pb;
    float rb;
    if (MODE == EV_A || MODE == EV_L) {
      Kb = K;
      pb = pi;
      rb = rho_i;
    } else {
      // state n of this particle: the sort of this evaluation took it from
      // slot perm[s] of the step's first sorted state
      Kb = at32(base.cell, eb);
      pb = at32(base.pv, eb);
      rb = at32(base.aux, eb).x;
    }
    float rn, rn_free, vx, vy, ox, oy, e_new = 0.0f;
    if constexpr (MODE == EV_L) {
      // leapfrog (scheme 1): merged kick v^(n+1/2) = v^(n-1/2) + (dt^(n-1) +
      // dt^n)/2 a^n, drift with the new velocity plus the XSPH correction,
      // internal energy by its rate (D); rho is the step's summed density
      const float kick = (float)(0.5 * (C.dt_prev + dt)), fdt = (float)dt;
      rn = rb;
      rn_free = rn;
      vx = pb.z + kick * acc.ax;
      vy = pb.w + kick * (acc.ay + P.gy);
      ox = pb.x + fdt * (vx + acc.Vx);
      oy = pb.y + fdt * (vy + acc.Vy);
      e_new = sb.e[s] + fdt * acc.D;
    } else {
      rn = rb + hdt * acc.D;
      rn_free = rn;
      if (rn < P.rho_lo) { rn = P.rho_lo; clamp_hit = true; }
      if (rn > P.rho_hi) { rn = P.rho_hi; clamp_hit = true; }
      vx = pb.z + hdt * acc.ax;
      vy = pb.w + hdt * (acc.ay + P.gy);
      ox = pb.x + hdt * (pi.z + acc.Vx);
      oy = pb.y + hdt * (pi.w + acc.Vy);
    }
    int cx, cy;
    cell_xy(P, Kb, cx, cy);
    renorm(ox, cx, P.dc);
    renorm(oy, cy, P.dc);
    // enforcement in FP64: hard walls, then radial pull-out from the disk
    double x = P.x_lo + (double)cx * P.dcd + (double)ox;
    double y = P.y_lo + (double)cy * P.dcd + (double)oy;
    if (d.tape_pos != nullptr) {  // pre-enforcement state for the reverse sweep
      const int fid = (int)id_i - P.id0;
      d.tape_pos[fid] = make_double2(x, y);
      d.tape_vel[fid] = make_float4(vx, vy, rb + hdt * acc.D, 0.0f);
    }
    const double k_free = (double)vx * vx + (double)vy * vy;
    bool moved = false;
    const double e = P.eps_wall;
    if (x < e) { x = e; vx = -vx; moved = true; }
    if (x > P.L - e) { x = P.L - e; vx = -vx; moved = true; }
    if (y < e) { y = e; vy = -vy; moved = true; }
    if (y > P.W - e) { y = P.W - e; vy = -vy; moved = true; }
    if (P.nd > 0) {
      // disk at the time of the new state (t + dt/2 or t + dt)
      double xd = C.xd_next, vd = C.vd_next;
      if (MODE == EV_A) {
        double ad;
        disk_at(P, C, C.t + 0.5 * dt, xd, vd, ad);
      }
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
      encode_axis(x, P.x_lo, P.dcd, P.inv_dcd, P.dc, P.ncx, cx, ox);
      encode_axis(y, P.y_lo, P.dcd, P.inv_dcd, P.dc, P.ncy, cy, oy);
    }
    cx = min(max(cx, 0), P.ncx - 1);
    cy = min(max(cy, 0), P.ncy - 1);
    const uint32_t Kn = (uint32_t)(P.cell_off + cy * P.ncx + cx);
    out.cell[s] = Kn;
    out.pv[s] = make_float4(ox, oy, vx, vy);
    out.aux[s] = make_float4(rn, 0.0f, 0.0f, 0.0f);
    out.id[s] = id_i;
    if constexpr (BATCH) out.inst[s] = (uint16_t)inst;
    if constexpr (MODE == EV_L) out.e[s] = e_new;
    newkey = Kn;
    vnew = fast_sqrt(vx * vx + vy * vy);
    if (!(rn == rn) || !(vnew <= 3.0e38f) || !(fabsf(e_new) <= 3.0e38f)) atomicOr(&clk[inst].bad, 1u);
    if constexpr (AUD && MODE == EV_B) {
      // the energy the enforcement and the density clamp add to the new state
      const double m = (double)h_m[threadIdx.x];
      if (moved) e_enf = 0.5 * m * ((double)vx * vx + (double)vy * vy - k_free);
      if (clamp_hit) e_clamp = m * (eos_e_el(P, (double)rn) - eos_e_el(P, (double)rn_free));
    }
  }
  if constexpr (AUD && MODE == EV_B) {
    // this block's audit terms, added to its own running sums (a fixed
    // order for every block, no atomics): the rates times dt, then the
    // enforcement and clamp energy
    const double m = lead ? (double)h_m[threadIdx.x] : 0.0;
    const double rate[4] = {m * h_aud[0][threadIdx.x], m * h_aud[1][threadIdx.x], m * h_aud[2][threadIdx.x],
                            m * h_aud[3][threadIdx.x]};
    double tot[6];
#pragma unroll
    for (int k = 0; k < 4; ++k) tot[k] = wave_sum(lead ? rate[k] : 0.0);
    tot[4] = wave_sum(e_enf);
    tot[5] = wave_sum(e_clamp);
    if (threadIdx.x == 0) {
      const double dt = clk[0].dt;
      double* a = d.audit_part + (size_t)blockIdx.x * 6;
#pragma unroll
      for (int k = 0; k < 4; ++k) a[k] += dt * tot[k];
      a[4] += tot[4];
      a[5] += tot[5];
    }
  }
  bucket_put_wave(d, next_fill, lead, newkey, (uint32_t)s);
  count_hits<BATCH>(clk, inst, clamp_hit, enf_hit);
  if (MODE == EV_L) {
    // as after a corrector: this block's max |v| of the new state for the
    // next step's dt (the clock pass has already closed this step)
    if constexpr (BATCH) {
      vmax_update<BATCH>(clk, inst, lead, vnew);
    } else {
      const float w = wave_max(lead ? vnew : 0.0f);
      if (threadIdx.x == 0) d.vmax_part[blockIdx.x] = w;
    }
  }
  if (MODE == EV_B) {
    if constexpr (BATCH) {
      vmax_update<BATCH>(clk, inst, lead, vnew);
    } else {
      // this block's max |v|, folded into the clock by the next first sort
      // (no atomics on one address from every wave)
      const float w = wave_max(lead ? vnew : 0.0f);
      if (threadIdx.x == 0) d.vmax_part[blockIdx.x] = w;
    }
    // work of the ring on the fluid over the step (fixed-order sum of the
    // per-ghost forces at t + dt/2) and the time of the new state; the first
    // wave of block i serves instance i
    for (int i = blockIdx.x; i < d.n_inst; i += gridDim.x) {
      if (threadIdx.x < 64) {
        const InstParams& Pi = d.prm[i];
        double f = 0.0;
        for (int k = (int)threadIdx.x; k < Pi.nd; k += 64) f += d.wb_part[i * WC_MAX_RING + k];
        f = wave_sum(f);
        if (threadIdx.x == 0) {
          Clock& Ci = clk[i];
          Ci.w_boundary += Ci.dt * f * (Pi.kin_mode == 2 && Ci.coupled ? Ci.v_work : Ci.vd);
          Ci.t_next = Ci.t + Ci.dt;
        }
      }
    }
  }
}

// Summation density of scheme 1 (eq. density-sum), in place on the sorted
// state: per fluid slot, the pair-sum machinery above sums |m_j| W_ij over
// the fluid and ghosts in support (the ring already at this step's time),
// the particle's own m_i W(0) is added, the result is clamped to the density
// band (counted), and the EOS with the internal energy fills (rho, P, c). A
// neighbour's aux is read only for its mass, which this pass does not
// change. count: add the clamp hits to the clock (0 for the test hooks).
template <bool BATCH, int VAR>
__global__ __launch_bounds__(PAIR_BLOCK) void k_dens(Dev d, Buf sb, int count) {
  __shared__ float4 uni[PAIR_BLOCK / 64][UCAP];
  __shared__ uint8_t lst[LCAP * PAIR_BLOCK];
  const int s0 = xcd_block(blockIdx.x, gridDim.x) * PAIR_SLOTS;
  const int q = (int)(threadIdx.x % PAIR_G);
  const int s = s0 + (int)(threadIdx.x / PAIR_G);
  const bool inr = s < d.n_slots;
  const int inst = inr ? inst_at<BATCH>(sb, s) : 0;
  uint32_t K = 0;
  float4 pi = make_float4(0, 0, 0, 0), ai = make_float4(0, 0, 0, 0);
  if (inr) {
    K = sb.cell[s];
    pi = sb.pv[s];
    ai = sb.aux[s];
  }
  const bool fluid = inr && ai.w > 0.0f;
  PairAcc acc = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
  AudAcc aud = {0.0f, 0.0f, 0.0f, 0.0f};
  pair_sums_wave<BATCH, false, VAR | 8>(d, sb, s, inst, K, fluid, pi, ai, q, uni[threadIdx.x >> 6],
                                        lst + threadIdx.x, acc, aud);
  const float sum = slot_sum(acc.D);
  bool clamp_hit = false;
  if (q == 0 && fluid) {
    const InstParams& P = d.prm[inst];
    float W0, F0;
    if constexpr ((VAR & 2) != 0) cubic_spline(P, 0.0f, W0, F0);
    else wendland(P, 0.0f, W0, F0);
    float rho = sum + ai.w * W0;
    if (rho < P.rho_lo) { rho = P.rho_lo; clamp_hit = true; }
    if (rho > P.rho_hi) { rho = P.rho_hi; clamp_hit = true; }
    float Pq, c;
    fluid_eos<true>(P, rho, Pq, c, sb.e[s]);
    sb.aux[s] = make_float4(rho, Pq, c, ai.w);
    if (!(rho == rho) || !(fabsf(Pq) <= 3.0e38f)) atomicOr(&d.clk[inst].bad, 1u);
  }
  if (count) count_hits<BATCH>(d.clk, inst, clamp_hit, false);
}

// The clock of a scheme-1 step (one wave per instance, after the ghost
// pass): dt from v_max (fluid of the stored state and ghosts) or the fixed
// table, the previous step's dt kept for the merged kick, the probe row's
// (t, dt), the disk at t + dt for the enforcement and the ring of the next
// step, the ring's work over the step (its x force at t times the disk
// velocity at t times dt, a fixed-order sum) and the new state's time.
__global__ __launch_bounds__(64) void k_clock_lf(Dev d) {
  const int i = blockIdx.x;
  const InstParams& P = d.prm[i];
  Clock& C = d.clk[i];
  double f = 0.0;
  for (int k = (int)threadIdx.x; k < P.nd; k += 64) f += d.wb_part[i * WC_MAX_RING + k];
  f = wave_sum(f);
  if (threadIdx.x != 0) return;
  const double dt = step_dt(d, P, C);
  C.dt_prev = C.dt;
  C.dt = dt;
  C.vmax_used = (double)__uint_as_float(C.vmax_bits);
  C.vmax_bits = 0u;
  const long long row = (long long)i * WC_HIST_CAP + (C.step % WC_HIST_CAP);
  d.hist_t[row] = C.t;
  d.hist_dt[row] = dt;
  double xn, vn, an;
  kinematics(P, C.t + dt, xn, vn, an);
  C.xd_next = xn;
  C.vd_next = vn;
  C.w_boundary += dt * f * C.vd;
  C.t_next = C.t + dt;
}

// Two-way coupled disk (kin_mode 2), one wave per instance between the
// second ghost pass and the second pair pass: the disk takes the reaction of
// the ring's x force on the fluid at t + dt/2 (the fixed-order sum of the
// per-ghost forces, the same sum as the boundary work), M dv/dt = -f, with a
// trapezoidal position. The state at t + dt places the ring and bounds the
// fluid of the new state; the step's mean velocity carries the boundary work.
__global__ __launch_bounds__(64) void k_disk(Dev d) {
  const int i = blockIdx.x;
  const InstParams& P = d.prm[i];
  Clock& C = d.clk[i];
  if (!(P.kin_mode == 2 && C.coupled)) return;
  double f = 0.0;
  for (int k = (int)threadIdx.x; k < P.nd; k += 64) f += d.wb_part[i * WC_MAX_RING + k];
  f = wave_sum(f);
  if (threadIdx.x == 0) {
    const double dt = C.dt, a1 = -f / P.disk_mass, v1 = C.vc + dt * a1;
    C.xd_next = C.xc + dt * 0.5 * (C.vc + v1);
    C.vd_next = v1;
    C.ac_next = a1;
    C.v_work = 0.5 * (C.vc + v1);
  }
}

// Disk centre, velocity and acceleration of instance i's newest state.
__global__ void k_disk_query(Dev d, int i, double* out) {
  if (threadIdx.x != 0) return;
  double x, v, a;
  disk_newest(d.prm[i], d.clk[i], x, v, a);
  out[0] = x;
  out[1] = v;
  out[2] = a;
}

// Buckets and v_max of a freshly loaded state (slots in any order); the
// disk ring is placed at the time of the state.
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
      const float4 pv = X.pv[s];
      v = fast_sqrt(pv.z * pv.z + pv.w * pv.w);
    } else if (local >= P.nf + P.nw) {
      double xc, vc, ac;
      disk_newest(P, d.clk[inst], xc, vc, ac);
      place_ring(d, P, inst, local - P.nf - P.nw, xc, X, s, fill_a(d));
    } else {
      bucket_put_wall(d, P, fill_a(d), X.cell[s], local - P.nf, (uint32_t)s);
    }
  }
  // fluid slots into their buckets, one counter update per run of equal keys
  bucket_put_wave(d, fill_a(d), fl, fl ? X.cell[s] : 0u, (uint32_t)s);
  vmax_update<BATCH>(d.clk, inst, fl, v);
  if (!BATCH && s < d.n_vpart) d.vmax_part[s] = 0.0f;  // the loaded state's max is in the clock
}

// FP64 diagnostics: partial sums over fixed chunks of each instance's slots
// (grid: WC_DIAG_BLOCKS x n_inst), then one fixed-order pass per instance.
__global__ __launch_bounds__(256) void k_diag_part(Dev d, Buf X, int sorted) {
  const int i = blockIdx.y, b = blockIdx.x;
  const InstParams& P = d.prm[i];
  int lo, hi;
  if (sorted) {
    lo = (int)d.start[P.cell_off];
    hi = (int)d.start[P.cell_off + P.ncell];
  } else {
    lo = P.id0;
    hi = P.id0 + P.nf + P.nw + P.nd;
  }
  const int chunk = (hi - lo + WC_DIAG_BLOCKS - 1) / WC_DIAG_BLOCKS;
  const int a = lo + b * chunk, e = min(hi, a + chunk);
  const double g = P.gammad, r0 = P.rho0d, B = P.Bd, m_plan = P.m_fluidd;
  const double rc = P.diag_rc, k1 = P.diag_k1, r0g1 = P.diag_r0g1, erc = P.diag_erc, inv_r0g = P.diag_inv_r0g;
  double M = 0, px = 0, py = 0, ke = 0, eel = 0, epot = 0, ncav = 0, bad = 0, eth = 0;
  for (int s = a + (int)threadIdx.x; s < e; s += 256) {
    const int local = (int)X.id[s] - P.id0;
    if (local < 0 || local >= P.nf) continue;
    // (axisymmetric: each particle weighs its ring mass 2 pi M / (2 pi))
    const double m = P.axisym ? 6.283185307179586 * d.mring[X.id[s]] : m_plan;
    const float4 pv = X.pv[s];
    const double r = (double)X.aux[s].x;
    const double ei = X.e ? (double)X.e[s] : 0.0;  // scheme 1: specific internal energy
    eth += m * ei;
    int cx, cy;
    cell_xy(P, X.cell[s], cx, cy);
    const double y = P.y_lo + (double)cy * P.dcd + (double)pv.y;
    const double u = pv.z, w = pv.w;
    M += m;
    px += m * u;
    py += m * w;
    ke += 0.5 * m * (u * u + w * w);
    if (P.eos_type == 1) {
      eel += m * mg_e_el(P, r);
      const double mu = r / r0 - 1.0;
      // (scheme 1: with the energy term gamma0 rho e of the tension branch)
      ncav += (mu < 0.0 && P.mg_Kd * mu + P.mg_g0d * r * ei <= P.p_cavd) ? 1.0 : 0.0;
    } else {
      const double rg1 = pow_gm1(r, g);
      // specific elastic energy of the Tait law, cutoff branch below rho_c
      eel += m * (r >= rc ? k1 * (rg1 - r0g1) + B * (1.0 / r - 1.0 / r0) : erc + P.p_cavd * (1.0 / rc - 1.0 / r));
      ncav += (B * (rg1 * r * inv_r0g - 1.0) <= P.p_cavd) ? 1.0 : 0.0;
    }
    epot += m * (-(double)P.gy) * y;
    if (!(r == r) || !(fabs(u) < 1e30) || !(fabs(w) < 1e30)) bad += 1.0;
  }
  const double v[WC_DIAG_PARTS] = {M, px, py, ke, eel, epot, ncav, bad, eth};
  __shared__ double ws[4][WC_DIAG_PARTS];
#pragma unroll
  for (int k = 0; k < WC_DIAG_PARTS; ++k) {
    const double x = wave_sum(v[k]);
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6][k] = x;
  }
  __syncthreads();
  if (threadIdx.x < WC_DIAG_PARTS) {
    const int k = threadIdx.x;
    d.diag_part[((long long)i * WC_DIAG_BLOCKS + b) * WC_DIAG_PARTS + k] =
        ((ws[0][k] + ws[1][k]) + ws[2][k]) + ws[3][k];
  }
}

__global__ __launch_bounds__(64) void k_diag_final(Dev d) {
  const int i = blockIdx.x;
  // fixed-order sum of the block partials: lane l adds blocks l, l + 64, ...
  // in order, then a butterfly over the wave
  static_assert(WC_DIAG_BLOCKS % 64 == 0, "whole waves of block partials");
  constexpr int NB = WC_DIAG_BLOCKS / 64;
  double part[NB][WC_DIAG_PARTS];  // every load in flight before the sums
#pragma unroll
  for (int j = 0; j < NB; ++j)
#pragma unroll
    for (int k = 0; k < WC_DIAG_PARTS; ++k)
      part[j][k] = d.diag_part[((long long)i * WC_DIAG_BLOCKS + threadIdx.x + 64 * j) * WC_DIAG_PARTS + k];
  double tot[WC_DIAG_PARTS];
#pragma unroll
  for (int k = 0; k < WC_DIAG_PARTS; ++k) {
    double v = 0.0;
#pragma unroll
    for (int j = 0; j < NB; ++j) v += part[j][k];
    tot[k] = wave_sum(v);
  }
  // energy audit: fixed-order sum of the pair blocks' running sums
  double aud[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  if (d.audit_part != nullptr) {
    for (int b = (int)threadIdx.x; b < d.n_vpart; b += 64)
#pragma unroll
      for (int k = 0; k < 6; ++k) aud[k] += d.audit_part[(size_t)b * 6 + k];
#pragma unroll
    for (int k = 0; k < 6; ++k) aud[k] = wave_sum(aud[k]);
  }
  if (threadIdx.x != 0) return;
  const InstParams& P = d.prm[i];
  Clock& C = d.clk[i];
  const long long row = C.diag_row++;
  double xd, vd, ad;
  disk_newest(P, C, xd, vd, ad);
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
#pragma unroll
  for (int k = 0; k < 6; ++k) o[15 + k] = aud[k];
  o[21] = tot[8];
  if (tot[7] > 0.0 || !(tot[3] == tot[3])) C.bad |= 1u;
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
#define NQ(n) (((n) + PAIR_SLOTS - 1) / PAIR_SLOTS)
int wc_pair_blocks(int n_slots) { return NQ(n_slots); }

// The ghost pass with the context's kernel.
template <int MODE, bool BATCH>
static void launch_ghost(const Dev& d, int n_gblk, const Buf& sb, hipStream_t st) {
  if (d.var & 2) k_ghost<MODE, BATCH, true><<<n_gblk, WC_GHOST_BLOCK, 0, st>>>(d, sb);
  else k_ghost<MODE, BATCH, false><<<n_gblk, WC_GHOST_BLOCK, 0, st>>>(d, sb);
}

// The pair pass of the context's scheme variant: bit 0 the quadratic AV
// term (some instance has beta > 0), bit 1 the cubic spline kernel; scheme 1
// (d.var bit 3) sums the internal-energy rate in place of the density rate.
template <int MODE, bool BATCH, bool AUD, int V4>
static void launch_pair_v(const Dev& d, const Buf& sb, const Buf& base, const Buf& out, hipStream_t st) {
  const dim3 g(NQ(d.n_slots)), b(PAIR_BLOCK);
  switch (d.var & 3) {
    case 0: k_pair<MODE, BATCH, AUD, V4 | 0><<<g, b, 0, st>>>(d, sb, base, out); break;
    case 1: k_pair<MODE, BATCH, AUD, V4 | 1><<<g, b, 0, st>>>(d, sb, base, out); break;
    case 2: k_pair<MODE, BATCH, AUD, V4 | 2><<<g, b, 0, st>>>(d, sb, base, out); break;
    default: k_pair<MODE, BATCH, AUD, V4 | 3><<<g, b, 0, st>>>(d, sb, base, out); break;
  }
}
template <int MODE, bool BATCH, bool AUD = false>
static void launch_pair(const Dev& d, const Buf& sb, const Buf& base, const Buf& out, hipStream_t st) {
  if constexpr (MODE == EV_L) launch_pair_v<MODE, BATCH, AUD, 4>(d, sb, base, out, st);
  else if constexpr (MODE == EV_EXPORT) {
    if (d.var & 8) launch_pair_v<MODE, BATCH, AUD, 4>(d, sb, base, out, st);
    else launch_pair_v<MODE, BATCH, AUD, 0>(d, sb, base, out, st);
  } else {
    launch_pair_v<MODE, BATCH, AUD, 0>(d, sb, base, out, st);
  }
}

// The summation-density pass (scheme 1) of the context's kernel.
template <bool BATCH>
static void launch_dens(const Dev& d, const Buf& sb, bool count, hipStream_t st) {
  const dim3 g(NQ(d.n_slots)), b(PAIR_BLOCK);
  if (d.var & 2) k_dens<BATCH, 2><<<g, b, 0, st>>>(d, sb, count ? 1 : 0);
  else k_dens<BATCH, 0><<<g, b, 0, st>>>(d, sb, count ? 1 : 0);
}

template <bool BATCH>
static void eval_sort(const Dev& d, hipStream_t st, int mode, const Buf& pre, const Buf& out) {
  const int nt = (d.n_cells + WC_SORT_TILE - 1) / WC_SORT_TILE + 1;  // the clock block, then the tiles
  if (d.var & 4) {
    if (mode == EV_A) k_sort<EV_A, BATCH, true><<<nt, SORT_BLOCK, 0, st>>>(d, pre, out);
    else if (mode == EV_B) k_sort<EV_B, BATCH, true><<<nt, SORT_BLOCK, 0, st>>>(d, pre, out);
    else if (mode == EV_L) k_sort<EV_L, BATCH, true><<<nt, SORT_BLOCK, 0, st>>>(d, pre, out);
    else k_sort<EV_EXPORT, BATCH, true><<<nt, SORT_BLOCK, 0, st>>>(d, pre, out);
  } else {
    if (mode == EV_A) k_sort<EV_A, BATCH, false><<<nt, SORT_BLOCK, 0, st>>>(d, pre, out);
    else if (mode == EV_B) k_sort<EV_B, BATCH, false><<<nt, SORT_BLOCK, 0, st>>>(d, pre, out);
    else if (mode == EV_L) k_sort<EV_L, BATCH, false><<<nt, SORT_BLOCK, 0, st>>>(d, pre, out);
    else k_sort<EV_EXPORT, BATCH, false><<<nt, SORT_BLOCK, 0, st>>>(d, pre, out);
  }
}

template <bool BATCH>
static void enqueue_step_t(const Dev& d, const Bufs& b, int n_gblk, bool two_way, bool audit, hipStream_t st) {
  eval_sort<BATCH>(d, st, EV_A, b.X, b.Y);
  launch_ghost<EV_A, BATCH>(d, n_gblk, b.Y, st);
  launch_pair<EV_A, BATCH>(d, b.Y, b.Y, b.Z, st);
  eval_sort<BATCH>(d, st, EV_B, b.Z, b.W);
  launch_ghost<EV_B, BATCH>(d, n_gblk, b.W, st);
  if (two_way) k_disk<<<d.n_inst, 64, 0, st>>>(d);
  if (!BATCH && audit) launch_pair<EV_B, false, true>(d, b.W, b.Y, b.X, st);
  else launch_pair<EV_B, BATCH>(d, b.W, b.Y, b.X, st);
}

// One leapfrog step (scheme 1) reading bucket set `set`: sort X into Y,
// summation density and EOS, ghosts and probes, the clock, then the pair
// pass with the update, back into X.
template <bool BATCH>
static void enqueue_lf_t(const Dev& d, const Bufs& b, int n_gblk, int set, hipStream_t st) {
  Dev dl = d;
  dl.lf_set = set;
  eval_sort<BATCH>(dl, st, EV_L, b.X, b.Y);
  launch_dens<BATCH>(dl, b.Y, true, st);
  launch_ghost<EV_L, BATCH>(dl, n_gblk, b.Y, st);
  k_clock_lf<<<d.n_inst, 64, 0, st>>>(dl);
  launch_pair<EV_L, BATCH>(dl, b.Y, b.Y, b.X, st);
}

void wc_enqueue_step(const Dev& d, const Bufs& b, int n_gblk, bool batch, bool two_way, bool audit,
                     hipStream_t st) {
  if (batch) enqueue_step_t<true>(d, b, n_gblk, two_way, false, st);
  else enqueue_step_t<false>(d, b, n_gblk, two_way, audit, st);
}

void wc_enqueue_step_lf(const Dev& d, const Bufs& b, int n_gblk, bool batch, int set, hipStream_t st) {
  if (batch) enqueue_lf_t<true>(d, b, n_gblk, set, st);
  else enqueue_lf_t<false>(d, b, n_gblk, set, st);
}

// Summation density of the export sort's state (scheme 1 test hooks).
void wc_enqueue_export_dens(const Dev& d, const Bufs& b, hipStream_t st) {
  launch_dens<false>(d, b.Y, false, st);
}

void wc_enqueue_disk_query(const Dev& d, int inst, double* out, hipStream_t st) {
  k_disk_query<<<1, 64, 0, st>>>(d, inst, out);
}

void wc_enqueue_init(const Dev& d, const Bufs& b, bool batch, hipStream_t st) {
  if (batch) k_init<true><<<NB(d.n_slots), WC_BLOCK, 0, st>>>(d, b.X);
  else k_init<false><<<NB(d.n_slots), WC_BLOCK, 0, st>>>(d, b.X);
}

void wc_enqueue_diag(const Dev& d, const Bufs& b, bool sorted, hipStream_t st) {
  k_diag_part<<<dim3(WC_DIAG_BLOCKS, d.n_inst), 256, 0, st>>>(d, b.X, sorted ? 1 : 0);
  k_diag_final<<<d.n_inst, 64, 0, st>>>(d);
}

// Eval-A sort of X into Y without advancing the clock (test hooks).
void wc_enqueue_export_sort(const Dev& d, const Bufs& b, bool batch, hipStream_t st) {
  if (batch) eval_sort<true>(d, st, EV_EXPORT, b.X, b.Y);
  else eval_sort<false>(d, st, EV_EXPORT, b.X, b.Y);
}

void wc_enqueue_export_ghosts(const Dev& d, const Bufs& b, int n_gblk, hipStream_t st) {
  launch_ghost<EV_EXPORT, false>(d, n_gblk, b.Y, st);
}

void wc_enqueue_export_pair(const Dev& d, const Bufs& b, hipStream_t st) {
  launch_pair<EV_EXPORT, false>(d, b.Y, b.Y, b.Z, st);
}

void wc_enqueue_pair_a(const Dev& d, const Bufs& b, bool batch, hipStream_t st) {
  if (batch) launch_pair<EV_A, true>(d, b.Y, b.Y, b.Z, st);
  else launch_pair<EV_A, false>(d, b.Y, b.Y, b.Z, st);
}

void wc_enqueue_neigh(const Dev& d, const Bufs& b, hipStream_t st) {
  k_neigh<<<NB(d.n_slots), WC_BLOCK, 0, st>>>(d, b.Y);
}

void wc_enqueue_eval(const Dev& d, const Bufs& b, int n_gblk, int mode, hipStream_t st) {
  if (mode == EV_A) {
    eval_sort<false>(d, st, EV_A, b.X, b.Y);
    launch_ghost<EV_A, false>(d, n_gblk, b.Y, st);
    launch_pair<EV_A, false>(d, b.Y, b.Y, b.Z, st);
  } else {
    eval_sort<false>(d, st, EV_B, b.Z, b.W);
    launch_ghost<EV_B, false>(d, n_gblk, b.W, st);
    launch_pair<EV_B, false>(d, b.W, b.Y, b.X, st);
  }
}
