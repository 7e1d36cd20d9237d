// wcsph_api.hip -- host runtime and C ABI of libwcsph.so.
//
// Builds the paper's problem set-up on the host in FP64 (fluid lattice with
// the disk interior removed, wall-ghost lattice, disk ring, probe points,
// cell grid), encodes it into the device layout, captures one
// predictor-corrector step into a HIP graph and replays it.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <mutex>
#include <vector>

#include "wcsph.h"
#include "wcsph_launch.h"

namespace {

struct WcError {
  wcsph_status st;
  std::string msg;
};

thread_local std::string g_create_error;

#define HC(call)                                                                           \
  do {                                                                                     \
    hipError_t e_ = (call);                                                                \
    if (e_ != hipSuccess)                                                                  \
      throw WcError{WCSPH_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_)};       \
  } while (0)

void require(bool ok, const std::string& msg) {
  if (!ok) throw WcError{WCSPH_E_INVALID, msg};
}

// Device scratch of the allocation-free entry point
// (wcsph_export_neighbour_lists_noalloc): a file-scope array of
// WC_SCRATCH_WORDS 32-bit words that every GPU the library runs on holds
// until the process ends. Host code never passes the array's name to a
// kernel or a copy: it uses the device address that hipGetSymbolAddress
// returns on each device, taken once per device at context creation.
#define WC_SCRATCH_WORDS (1u << 20)  // 4 MiB
#define WC_MAX_DEVICES 64
static __device__ __align__(256) uint32_t scratch[WC_SCRATCH_WORDS];
std::mutex g_scratch_mu;
void* g_scratch_ptr[WC_MAX_DEVICES] = {};

// The scratch address on the current device (looked up once per device).
void* scratch_address() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= WC_MAX_DEVICES)
    throw WcError{WCSPH_E_HIP, "no current HIP device for the scratch array"};
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr)
      throw WcError{WCSPH_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e)};
    g_scratch_ptr[dev] = p;
  }
  return g_scratch_ptr[dev];
}

// Host-side geometry of one instance (FP64).
struct HostInst {
  std::vector<double> fx, fy, frho;  // fluid lattice (id order)
  std::vector<double> wx, wy;        // wall ghosts (id order)
  int nd = 0;
};

}  // namespace

struct wcsph_ctx {
  std::string err;
  uint32_t* nb_ids = nullptr;  // neighbour-list export buffer (allocated on first use)
  uint32_t* scratch = nullptr; // this context's device's file-scope scratch array (set at creation)
  hipStream_t st = nullptr;
  wcsph_allocator al{};
  bool custom_alloc = false;
  std::vector<void*> blocks;
  bool batch = false;
  int n_inst = 0;
  std::vector<wcsph_params> pin;
  std::vector<InstParams> hp;
  std::vector<HostInst> geo;
  long long n_fluid = 0;
  int n_slots = 0, n_cells = 0, n_ghost = 0, n_gblk = 0;
  int diag_every = 0;
  Dev d{};
  Bufs b{};
  InstParams* d_prm = nullptr;
  Clock* d_clk = nullptr;
  uint32_t* d_wallcount = nullptr;
  uint32_t* d_wall_tot = nullptr;  // static wall-ghost entries per sort tile
  double* d_kin_tab = nullptr;      // per instance: WC_KIN_ROWS rows (t, x, v, a) of a tabulated disk motion
  size_t n_tiles = 0;
  uint32_t* d_gslot_save = nullptr;
  std::vector<uint32_t> h_wallcount, h_wrank;
  std::vector<int4> h_gblk;
  hipGraph_t graph = nullptr;       // one step
  hipGraphExec_t gexec = nullptr;
  hipGraph_t graph_k = nullptr;     // steps_k steps and a diagnostic record
  hipGraphExec_t gexec_k = nullptr;
  // scheme 1: the same two graphs starting on bucket set b (the ones above start on set a)
  hipGraph_t graph1 = nullptr, graph_k1 = nullptr;
  hipGraphExec_t gexec1 = nullptr, gexec_k1 = nullptr;
  int scheme = 0;  // 0 predictor-corrector, 1 leapfrog with summation density
  int lf_set = 0;  // scheme 1: the bucket set the next step's sort reads
  int steps_k = 0;
  long long steps = 0;
  std::vector<long long> hist_read, diag_rows, diag_read;
  double* d_dt = nullptr;
  size_t d_dt_cap = 0;
  double* d_disk = nullptr;  // disk state query output (3 doubles)
  bool audit = false;        // energy audit in the second pair pass (single instance)
  bool dead = false;
  // reverse sweep
  struct Adj {
    bool fwd_done = false;
    int n_steps = 0, ckpt = 0, n_seg = 0;
    long long step0 = 0;
    std::vector<double> t, dt;         // time and step of every forward step
    std::vector<char*> ckpt_dev;       // state at each segment start, then the end state
    size_t ckpt_bytes = 0;
    int tape_steps = 0;                // taped steps allocated
    bool taped = false;                // the forward taped the whole run (no replay)
    std::vector<hipGraph_t> tg_graph;  // the taping forward of tg_n steps, in graphs of a few steps
    std::vector<hipGraphExec_t> tg_exec;
    int tg_n = 0;
    Dev tg_dev{};                      // ... captured for this device state and these buffers
    Bufs tg_bufs{};
    std::vector<TapeEval> tA, tB;
    std::vector<double2*> pA, pB;
    std::vector<float4*> vA, vB;
    AdjPtrs a{};
    float *L0 = nullptr, *L1 = nullptr, *Ls = nullptr;
    int nblk = 0;
    double J = 0.0;
  } adj;
};

namespace {

void* dalloc(wcsph_ctx* c, size_t bytes) {
  bytes = std::max<size_t>(bytes, 256);
  void* p = nullptr;
  if (c->custom_alloc) {
    p = c->al.alloc(bytes, (void*)c->st, c->al.user);
  } else if (hipMalloc(&p, bytes) != hipSuccess) {
    p = nullptr;
  }
  if (!p) throw WcError{WCSPH_E_OOM, "device allocation of " + std::to_string(bytes) + " bytes failed"};
  c->blocks.push_back(p);
  return p;
}

template <class T>
T* dalloc_n(wcsph_ctx* c, size_t n) {
  return static_cast<T*>(dalloc(c, n * sizeof(T)));
}

float cell_edge(const wcsph_params& p) {
  const double two_h = 2.0 * p.h_over_dx * p.dx;
  if (p.cell_size > 0) return (float)p.cell_size;
  float c = (float)two_h;
  if ((double)c < two_h) c = std::nextafter(c, INFINITY);
  return c;
}

void validate(const wcsph_params& p) {
  require(p.dx > 0 && std::isfinite(p.dx), "dx must be positive");
  require(p.L > 0 && p.W > 0, "L and W must be positive");
  require(p.h_over_dx >= 1.0 && p.h_over_dx <= 2.0, "h_over_dx must lie in [1, 2]");
  const double two_h = 2.0 * p.h_over_dx * p.dx;
  if (p.cell_size > 0) {
    require((double)(float)p.cell_size == p.cell_size, "cell_size must be a float32 value");
    require(p.cell_size >= two_h, "cell_size must be >= 2h");
  }
  require(p.rho0 > 0 && p.c0 > 0 && p.gamma > 1.0, "rho0, c0 must be positive and gamma > 1");
  require(p.p_cav <= 0, "p_cav must be <= 0");
  require(p.alpha >= 0 && p.delta >= 0 && p.eps_xsph >= 0 && p.mu_dyn >= 0 && p.eta2 > 0,
          "scheme coefficients must be non-negative (eta2 > 0)");
  require(p.cfl > 0 && p.cfl <= 1.0, "cfl must lie in (0, 1]");
  require(p.rho_lo > 0 && p.rho_hi > p.rho_lo, "density band must satisfy 0 < rho_lo < rho_hi");
  require(p.eps_wall >= 0 && p.eps_wall < 0.5 * p.dx, "eps_wall must lie in [0, dx/2)");
  require(p.ghost_layers >= 1 && p.ghost_layers <= 8, "ghost_layers must lie in [1, 8]");
  require(p.n_disk_ghosts >= 0 && p.n_disk_ghosts <= WC_MAX_RING,
          "n_disk_ghosts must lie in [0, 256]");
  require(p.ghost_rho_mode == 0 || p.ghost_rho_mode == 1, "ghost_rho_mode must be 0 or 1");
  require(p.init_mode == 0 || p.init_mode == 1, "init_mode must be 0 or 1");
  require(p.disk_R >= 0, "disk_R must be >= 0");
  require(p.axisym == 0 || p.axisym == 1, "axisym must be 0 or 1");
  if (p.axisym) {
    require(p.scheme == 0, "the axisymmetric form takes scheme 0 only");
    require(p.gravity_y == 0.0, "the axisymmetric form needs gravity_y = 0");
    require(p.audit == 0, "the axisymmetric form does not take the energy audit");
    if (p.disk_R > 0) require(p.disk_y0 == 0.0, "the axisymmetric sphere's centre must lie on the axis (disk_y0 = 0)");
  }
  if (p.disk_R > 0) {
    // (axisymmetric: the sphere straddles the axis, the box holds its upper half)
    const double y_lo = p.axisym ? -p.disk_R : 0.0;
    require(p.disk_x0 - p.disk_R >= -1e-12 && p.disk_x0 + p.disk_R <= p.L + 1e-12 &&
                p.disk_y0 - p.disk_R >= y_lo - 1e-12 && p.disk_y0 + p.disk_R <= p.W + 1e-12,
            "disk must lie inside the channel");
    require(p.kin_t_ramp > 0 && p.kin_v0 >= 0 && p.kin_coef >= 0, "kinematics coefficients invalid");
  }
  require(p.kin_mode >= 0 && p.kin_mode <= 3, "kin_mode must be 0, 1, 2 or 3");
  if (p.disk_R > 0 && p.kin_mode == 2)
    require(p.disk_mass > 0 && std::isfinite(p.disk_mass), "a two-way coupled disk needs disk_mass > 0");
  require(p.n_probes >= 0 && p.n_probes <= WCSPH_MAX_PROBES, "n_probes must lie in [0, 16]");
  const double m = p.ghost_layers * p.dx;
  for (int k = 0; k < p.n_probes; ++k)
    require(p.probe_xy[2 * k] >= -m && p.probe_xy[2 * k] <= p.L + m && p.probe_xy[2 * k + 1] >= -m &&
                p.probe_xy[2 * k + 1] <= p.W + m,
            "probe outside the grid");
  require(p.diag_every >= 0, "diag_every must be >= 0");
  require(p.audit == 0 || p.audit == 1, "audit must be 0 or 1");
  require(p.beta >= 0 && std::isfinite(p.beta), "beta must be finite and >= 0");
  require(p.kernel_type == 0 || p.kernel_type == 1, "kernel_type must be 0 (Wendland C2) or 1 (cubic spline)");
  require(p.scheme == 0 || p.scheme == 1, "scheme must be 0 (predictor-corrector) or 1 (leapfrog, summation density)");
  if (p.scheme == 1) {
    require(p.kin_mode != 2, "scheme 1 does not take the two-way coupled disk (kin_mode 2)");
    require(p.audit == 0, "scheme 1 does not take the energy audit");
    require(p.mg_a >= 0.0 && std::isfinite(p.mg_a), "mg_a must be finite and >= 0");
  }
  require(p.eos_type == 0 || p.eos_type == 1, "eos_type must be 0 (Tait) or 1 (Mie-Grueneisen)");
  if (p.eos_type == 1)
    require(p.mg_s1 >= 1.0 && p.mg_gamma0 >= 0.0 && p.mg_gamma0 < 2.0 && p.mg_mu_max > 0.0 &&
                (p.mg_s1 - 1.0) * p.mg_mu_max < 0.9 && std::isfinite(p.mg_s1 + p.mg_gamma0 + p.mg_mu_max),
            "Mie-Grueneisen parameters need S1 >= 1, 0 <= gamma0 < 2, mu_max > 0, (S1 - 1) mu_max < 0.9");
  const long long nx = std::llround(p.L / p.dx), ny = std::llround(p.W / p.dx);
  require(nx >= 1 && ny >= 1 && nx * ny < (1ll << 28), "lattice size out of range");
}

// Density at pressure q >= 0 on the instance's EOS (the hydrostatic start):
// the Tait inverse, or for the Mie-Grueneisen law the root in [0, 1/b) of
// s (1 - b mu)^2 = mu (1 + k1 mu), s = q / (rho0 C^2), capped at mu_max.
double eos_density(const wcsph_params& p, double B, double q) {
  if (p.eos_type == 0) return p.rho0 * std::pow(1.0 + q / B, 1.0 / p.gamma);
  const double s = q / (p.rho0 * p.c0 * p.c0), b = p.mg_s1 - 1.0, k1 = 1.0 - 0.5 * p.mg_gamma0;
  const double mu = 2.0 * s / ((1.0 + 2.0 * b * s) + std::sqrt(1.0 + 4.0 * s * (b + k1)));
  return p.rho0 * (1.0 + std::min(mu, p.mg_mu_max));
}

// Problem set-up of one instance: fluid lattice ((i+1/2)dx, (j+1/2)dx) with
// id = j nx + i and the disk interior removed; wall ghosts continuing the
// lattice ghost_layers deep around the box (j outer); the disk ring.
HostInst build_geometry(const wcsph_params& p) {
  HostInst g;
  const int nx = (int)std::lround(p.L / p.dx), ny = (int)std::lround(p.W / p.dx);
  const double B = p.rho0 * p.c0 * p.c0 / p.gamma;
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      const double x = (i + 0.5) * p.dx, y = (j + 0.5) * p.dx;
      if (p.disk_R > 0) {
        const double ux = x - p.disk_x0, uy = y - p.disk_y0;
        if (ux * ux + uy * uy < p.disk_R * p.disk_R) continue;
      }
      double r = p.rho0;
      if (p.init_mode == 1) r = eos_density(p, B, p.rho0 * std::fabs(p.gravity_y) * (p.W - y));
      g.fx.push_back(x);
      g.fy.push_back(y);
      g.frho.push_back(r);
    }
  const int Lg = p.ghost_layers;
  for (int j = -Lg; j < ny + Lg; ++j)
    for (int i = -Lg; i < nx + Lg; ++i) {
      if (i >= 0 && i < nx && j >= 0 && j < ny) continue;
      g.wx.push_back((i + 0.5) * p.dx);
      g.wy.push_back((j + 0.5) * p.dx);
    }
  g.nd = p.disk_R > 0 ? p.n_disk_ghosts : 0;
  return g;
}

// Scheme 1 particle mass: rho0 over the kernel sum of the square lattice of
// spacing dx (every lattice point within 2h of a particle, itself included),
// so that the undisturbed lattice sums to rho0 (Density Summation).
double lattice_mass(const wcsph_params& p) {
  const double h = p.h_over_dx * p.dx;
  double S = 0.0;
  for (int j = -4; j <= 4; ++j)
    for (int i = -4; i <= 4; ++i) {
      const double q = std::sqrt((double)(i * i + j * j)) * p.dx / h;
      if (q >= 2.0) continue;
      if (p.kernel_type == 1) {
        const double sg = 10.0 / (7.0 * M_PI * h * h);
        S += q <= 1.0 ? sg * (1.0 - 1.5 * q * q + 0.75 * q * q * q) : sg * 0.25 * (2.0 - q) * (2.0 - q) * (2.0 - q);
      } else {
        const double u = 1.0 - 0.5 * q;
        S += 7.0 / (4.0 * M_PI * h * h) * u * u * u * u * (2.0 * q + 1.0);
      }
    }
  return p.rho0 / S;
}

InstParams derive(const wcsph_params& p) {
  InstParams q;
  std::memset(&q, 0, sizeof q);
  const double h = p.h_over_dx * p.dx;
  q.dc = cell_edge(p);
  q.dcd = (double)q.dc;
  q.inv_dcd = 1.0 / q.dcd;
  q.x_lo = -p.ghost_layers * p.dx;
  q.y_lo = -p.ghost_layers * p.dx;
  q.ncx = (int)std::ceil((p.L + 2.0 * p.ghost_layers * p.dx) / q.dcd);
  q.ncy = (int)std::ceil((p.W + 2.0 * p.ghost_layers * p.dx) / q.dcd);
  q.ncell = q.ncx * q.ncy;
  q.h = (float)h;
  q.inv_h = (float)(1.0 / h);
  q.four_h2 = (float)(4.0 * h * h);
  q.sigma = (float)(7.0 / (4.0 * M_PI * h * h));
  q.fgrad = (float)(35.0 / (4.0 * M_PI * h * h * h * h));
  q.eta2h2 = (float)(p.eta2 * h * h);
  const double B = p.rho0 * p.c0 * p.c0 / p.gamma;
  q.rho0 = (float)p.rho0;
  q.c0 = (float)p.c0;
  q.B = (float)B;
  q.p_cav = (float)p.p_cav;
  q.alpha = (float)p.alpha;
  q.beta2h2 = (float)(2.0 * p.beta * h * h);
  q.kernel_type = p.kernel_type;
  q.kc_sigma = (float)(10.0 / (7.0 * M_PI * h * h));
  q.kc_a = (float)(10.0 / (7.0 * M_PI * h * h * h * h));
  q.eps_xsph = (float)p.eps_xsph;
  q.gy = (float)p.gravity_y;
  q.two_delta_h_c0 = (float)(2.0 * p.delta * h * p.c0);
  q.four_nu0 = (float)(4.0 * p.mu_dyn / p.rho0);
  q.delta = (float)p.delta;
  q.two_h_c0 = (float)(2.0 * h * p.c0);
  const double m_part = p.scheme == 1 ? lattice_mass(p) : p.rho0 * p.dx * p.dx;
  q.m_fluid = (float)m_part;
  q.m_wall = (float)m_part;
  q.m_disk = p.n_disk_ghosts > 0 ? (float)(m_part / p.dx * 2.0 * M_PI * p.disk_R / p.n_disk_ghosts) : 0.0f;
  q.scheme = p.scheme;
  q.axisym = p.axisym;
  q.r_mind = 0.5 * p.dx;
  q.r_min = (float)q.r_mind;
  q.mg_a = (float)p.mg_a;
  q.mg_g0 = (float)p.mg_gamma0;
  q.mg_ad = p.mg_a;
  q.mg_g0d = p.mg_gamma0;
  q.rho_lo = (float)(p.rho_lo * p.rho0);
  q.rho_hi = (float)(p.rho_hi * p.rho0);
  q.inv_rho0c02 = (float)(1.0 / (p.rho0 * p.c0 * p.c0));
  q.c_exp = (float)(0.5 * (p.gamma - 1.0));
  q.gamma = (float)p.gamma;
  q.inv_gamma = (float)(1.0 / p.gamma);
  q.ghost_rho_mode = p.ghost_rho_mode;
  q.eos_type = p.eos_type;
  {
    const double K = p.rho0 * p.c0 * p.c0, b = p.mg_s1 - 1.0, k1 = 1.0 - 0.5 * p.mg_gamma0, m = p.mg_mu_max;
    q.mg_K = (float)K;
    q.mg_k1 = (float)k1;
    q.mg_b = (float)b;
    q.mg_mu_max = (float)m;
    q.mg_Kd = K;
    q.mg_k1d = k1;
    q.mg_bd = b;
    q.mg_mu_maxd = m;
    q.mg_mu_cavd = p.p_cav / K;
    q.mg_p_capd = K * m * (1.0 + k1 * m) / ((1.0 - b * m) * (1.0 - b * m));
  }
  q.L = p.L;
  q.W = p.W;
  q.eps_wall = p.eps_wall;
  q.R = p.disk_R;
  q.disk_x0 = p.disk_x0;
  q.disk_y0 = p.disk_y0;
  q.disk_mass = p.disk_mass;
  q.cfl = p.cfl;
  q.hd = h;
  q.c0d = p.c0;
  q.Bd = B;
  q.rho0d = p.rho0;
  q.gammad = p.gamma;
  q.p_cavd = p.p_cav;
  q.m_fluidd = m_part;
  {
    const double g = p.gamma, r0 = p.rho0;
    q.diag_rc = r0 * std::pow(1.0 + p.p_cav / B, 1.0 / g);
    q.diag_k1 = B / ((g - 1.0) * std::pow(r0, g));
    q.diag_r0g1 = std::pow(r0, g - 1.0);
    q.diag_erc = B * ((std::pow(q.diag_rc, g - 1.0) - q.diag_r0g1) / ((g - 1.0) * std::pow(r0, g)) + 1.0 / q.diag_rc -
                      1.0 / r0);
    q.diag_inv_r0g = 1.0 / std::pow(r0, g);
  }
  q.kin_mode = p.kin_mode;
  q.kin_v0 = p.kin_v0;
  q.kin_t_ramp = p.kin_t_ramp;
  q.kin_coef = p.kin_coef;
  return q;
}

void encode(const InstParams& q, double x, double y, uint32_t& key, float& ox, float& oy) {
  auto axis = [&](double v, double lo, int n, int& c, float& o) {
    const double u = v - lo;
    c = (int)std::floor(u / q.dcd);
    c = std::min(std::max(c, 0), n - 1);
    o = (float)(u - (double)c * q.dcd);
    if (o >= q.dc && c < n - 1) {
      o -= q.dc;
      c += 1;
    }
  };
  int cx, cy;
  axis(x, q.x_lo, q.ncx, cx, ox);
  axis(y, q.y_lo, q.ncy, cy, oy);
  key = (uint32_t)(q.cell_off + cy * q.ncx + cx);
}

void decode(const InstParams& q, uint32_t key, float ox, float oy, double& x, double& y) {
  const int local = (int)key - q.cell_off;
  const int cy = local / q.ncx, cx = local - cy * q.ncx;
  x = q.x_lo + (double)cx * q.dcd + (double)ox;
  y = q.y_lo + (double)cy * q.dcd + (double)oy;
}

void alloc_buf(wcsph_ctx* c, Buf& b) {
  const size_t n = c->n_slots;
  b.cell = dalloc_n<uint32_t>(c, n);
  b.id = dalloc_n<uint32_t>(c, n);
  b.pv = dalloc_n<float4>(c, n);
  b.aux = dalloc_n<float4>(c, n);
  b.inst = c->batch ? dalloc_n<uint16_t>(c, n) : nullptr;
}

void sync(wcsph_ctx* c) { HC(hipStreamSynchronize(c->st)); }

// The validity flags of instance inst's state (after a sync): 1 non-finite
// state (this instance); on instance 0 for the whole context: 4 corrupted
// permutation, 8 a cell holds more than WC_BUCKET particles. Sets the error text and returns true when
// any is set; the outputs already written stay for inspection.
bool state_invalid(wcsph_ctx* ctx, int inst) {
  Clock k, k0;
  HC(hipMemcpy(&k, ctx->d_clk + inst, sizeof k, hipMemcpyDeviceToHost));
  HC(hipMemcpy(&k0, ctx->d_clk, sizeof k0, hipMemcpyDeviceToHost));
  const unsigned bad = k.bad | (k0.bad & ~1u);
  if (!bad) return false;
  std::string m;
  if (bad & 1u) m += " non-finite or escaped particle;";
  if (bad & 4u) m += " corrupted cell-list permutation;";
  if (bad & 8u) m += " more than " + std::to_string(WC_BUCKET) + " particles in one cell;";
  ctx->err = "state invalid (flags " + std::to_string(bad) + "):" + m;
  return true;
}

// Refill the buckets of the next sort from the state in X (after the state,
// the clocks or the disk law changed from the host).
void arm_counts(wcsph_ctx* c) {
  HC(hipMemcpyAsync(c->d.count, c->d_wallcount, (size_t)c->n_cells * 4, hipMemcpyDeviceToDevice, c->st));
  HC(hipMemcpyAsync(c->d.tot_a, c->d_wall_tot, c->n_tiles * 4, hipMemcpyDeviceToDevice, c->st));
}
void rearm(wcsph_ctx* c) {
  arm_counts(c);
  wc_enqueue_init(c->d, c->b, c->batch, c->st);
  HC(hipGetLastError());
  c->lf_set = 0;  // bucket set a now holds the next sort's entries
}

// Write the set-up (or a given fluid state for instance 0) into X in id
// order, re-arm the sort counters and reset the clocks.
void upload_state(wcsph_ctx* c, double t0, const double* fx, const double* fy, const double* fvx,
                  const double* fvy, const double* frho) {
  const size_t n = c->n_slots;
  std::vector<uint32_t> cell(n), id(n);
  std::vector<float4> pv(n), aux(n);
  std::vector<uint16_t> inst(n);
  std::vector<uint32_t> gslot(c->n_ghost);
  for (int i = 0; i < c->n_inst; ++i) {
    const InstParams& q = c->hp[i];
    const HostInst& g = c->geo[i];
    const wcsph_params& p = c->pin[i];
    for (int k = 0; k < q.nf; ++k) {
      const size_t s = q.id0 + k;
      const bool given = fx != nullptr && i == 0;
      const double x = given ? fx[k] : g.fx[k], y = given ? fy[k] : g.fy[k];
      float ox, oy;
      encode(q, x, y, cell[s], ox, oy);
      pv[s] = make_float4(ox, oy, given ? (float)fvx[k] : 0.0f, given ? (float)fvy[k] : 0.0f);
      aux[s] = make_float4(given ? (float)frho[k] : (float)g.frho[k], 0, 0, 0);
      id[s] = (uint32_t)s;
      inst[s] = (uint16_t)i;
    }
    for (int k = 0; k < q.nw; ++k) {
      const size_t s = q.id0 + q.nf + k;
      float ox, oy;
      encode(q, g.wx[k], g.wy[k], cell[s], ox, oy);
      pv[s] = make_float4(ox, oy, 0, 0);
      aux[s] = make_float4((float)p.rho0, 0, 0, 0);
      id[s] = (uint32_t)s;
      inst[s] = (uint16_t)i;
      gslot[q.gmap0 + k] = (uint32_t)s;
    }
    for (int k = 0; k < q.nd; ++k) {
      const size_t s = q.id0 + q.nf + q.nw + k;
      float ox, oy;
      encode(q, p.disk_x0, p.disk_y0, cell[s], ox, oy);  // placed by the first evaluation
      pv[s] = make_float4(ox, oy, 0, 0);
      aux[s] = make_float4((float)p.rho0, 0, 0, 0);
      id[s] = (uint32_t)s;
      inst[s] = (uint16_t)i;
      gslot[q.gmap0 + q.nw + k] = (uint32_t)s;
    }
  }
  HC(hipMemcpyAsync(c->b.X.cell, cell.data(), n * 4, hipMemcpyHostToDevice, c->st));
  HC(hipMemcpyAsync(c->b.X.id, id.data(), n * 4, hipMemcpyHostToDevice, c->st));
  HC(hipMemcpyAsync(c->b.X.pv, pv.data(), n * 16, hipMemcpyHostToDevice, c->st));
  HC(hipMemcpyAsync(c->b.X.aux, aux.data(), n * 16, hipMemcpyHostToDevice, c->st));
  if (c->b.X.e) HC(hipMemsetAsync(c->b.X.e, 0, n * 4, c->st));  // scheme 1: no internal energy yet
  if (c->batch) HC(hipMemcpyAsync(c->b.X.inst, inst.data(), n * 2, hipMemcpyHostToDevice, c->st));
  HC(hipMemcpyAsync(c->d.gslot, gslot.data(), gslot.size() * 4, hipMemcpyHostToDevice, c->st));
  arm_counts(c);
  std::vector<Clock> clk(c->n_inst);
  for (auto& k : clk) {
    std::memset(&k, 0, sizeof k);
    k.t = t0;
    k.t_next = t0;
    k.step = -1;
  }
  HC(hipMemcpyAsync(c->d_clk, clk.data(), clk.size() * sizeof(Clock), hipMemcpyHostToDevice, c->st));
  if (c->d.audit_part)
    HC(hipMemsetAsync(c->d.audit_part, 0, (size_t)c->d.n_vpart * 6 * sizeof(double), c->st));
  wc_enqueue_init(c->d, c->b, c->batch, c->st);
  HC(hipGetLastError());
  c->steps = 0;
  for (int i = 0; i < c->n_inst; ++i) {
    c->hist_read[i] = 0;
    c->diag_rows[i] = 0;
    c->diag_read[i] = 0;
  }
  wc_enqueue_diag(c->d, c->b, false, c->st);
  HC(hipGetLastError());
  for (int i = 0; i < c->n_inst; ++i) c->diag_rows[i] = 1;
  sync(c);
}

void drop_graphs(wcsph_ctx* c) {
  for (hipGraphExec_t* e : {&c->gexec, &c->gexec_k, &c->gexec1, &c->gexec_k1}) {
    if (*e) hipGraphExecDestroy(*e);
    *e = nullptr;
  }
  for (hipGraph_t* g : {&c->graph, &c->graph_k, &c->graph1, &c->graph_k1}) {
    if (*g) hipGraphDestroy(*g);
    *g = nullptr;
  }
}

// Some instance has a two-way coupled disk: the step launches the disk update.
bool two_way(const wcsph_ctx* c) {
  for (const InstParams& q : c->hp)
    if (q.kin_mode == 2 && q.nd > 0) return true;
  return false;
}

// Capture the step graphs: one step, and diag_every steps followed by the
// diagnostic record (launched when the step count is a multiple of
// diag_every), so that consecutive steps run without host round trips.
// One step of the context's scheme; a leapfrog step reads bucket set `set`.
void enqueue_one_step(wcsph_ctx* c, int set) {
  if (c->scheme == 1) wc_enqueue_step_lf(c->d, c->b, c->n_gblk, c->batch, set, c->st);
  else wc_enqueue_step(c->d, c->b, c->n_gblk, c->batch, two_way(c), c->audit, c->st);
}
void capture_pair(wcsph_ctx* c, int set, hipGraph_t* g1, hipGraphExec_t* e1, hipGraph_t* gk, hipGraphExec_t* ek) {
  hipGraph_t g = nullptr;
  HC(hipStreamBeginCapture(c->st, hipStreamCaptureModeThreadLocal));
  enqueue_one_step(c, set);
  HC(hipStreamEndCapture(c->st, &g));
  *g1 = g;
  HC(hipGraphInstantiate(e1, g, nullptr, nullptr, 0));
  g = nullptr;
  HC(hipStreamBeginCapture(c->st, hipStreamCaptureModeThreadLocal));
  for (int k = 0; k < c->steps_k; ++k) enqueue_one_step(c, set ^ (k & 1));
  if (c->diag_every > 0) wc_enqueue_diag(c->d, c->b, true, c->st);
  HC(hipStreamEndCapture(c->st, &g));
  *gk = g;
  HC(hipGraphInstantiate(ek, g, nullptr, nullptr, 0));
}
void capture(wcsph_ctx* c) {
  drop_graphs(c);
  c->steps_k = c->diag_every > 0 ? c->diag_every : 10;
  capture_pair(c, 0, &c->graph, &c->gexec, &c->graph_k, &c->gexec_k);
  // scheme 1 alternates the bucket sets from step to step
  if (c->scheme == 1) capture_pair(c, 1, &c->graph1, &c->gexec1, &c->graph_k1, &c->gexec_k1);
}

void build(wcsph_ctx* c, const wcsph_params* params, int n_inst) {
  c->n_inst = n_inst;
  c->scheme = params[0].scheme;
  for (int i = 1; i < n_inst; ++i)
    require(params[i].scheme == c->scheme, "every instance of a batch must use the same scheme");
  c->pin.assign(params, params + n_inst);
  c->diag_every = params[0].diag_every;
  int id0 = 0, gmap0 = 0, cell_off = 0;
  for (int i = 0; i < n_inst; ++i) {
    const wcsph_params& p = params[i];
    HostInst g = build_geometry(p);
    InstParams q = derive(p);
    q.nf = (int)g.fx.size();
    q.nw = (int)g.wx.size();
    q.nd = g.nd;
    q.id0 = id0;
    q.gmap0 = gmap0;
    q.cell_off = cell_off;
    q.n_probes = p.n_probes;
    for (int k = 0; k < p.n_probes; ++k) {
      encode(q, p.probe_xy[2 * k], p.probe_xy[2 * k + 1], q.probe_cell[k], q.probe_ox[k], q.probe_oy[k]);
    }
    id0 += q.nf + q.nw + q.nd;
    gmap0 += q.nw + q.nd;
    cell_off += q.ncell;
    require((long long)id0 < (1ll << 28) && (long long)cell_off < (1ll << 30), "problem too large");
    c->n_fluid += q.nf;
    c->hp.push_back(q);
    c->geo.push_back(std::move(g));
  }
  c->n_slots = id0;
  c->n_ghost = gmap0;
  c->n_cells = cell_off;
  // static wall-ghost occupancy and bucket ranks; ghost-kernel block table
  c->h_wallcount.assign(c->n_cells, 0);
  c->h_wrank.assign(c->n_ghost, 0);
  for (int i = 0; i < n_inst; ++i) {
    const InstParams& q = c->hp[i];
    for (int k = 0; k < q.nw; ++k) {
      uint32_t key;
      float ox, oy;
      encode(q, c->geo[i].wx[k], c->geo[i].wy[k], key, ox, oy);
      c->h_wrank[q.gmap0 + k] = c->h_wallcount[key]++;
    }
    const int gq = WC_GHOST_BLOCK / WC_GHOST_LANES;  // ghosts or probes per block
    for (int g0 = 0; g0 < q.nw; g0 += gq) c->h_gblk.push_back(make_int4(i, g0, std::min(gq, q.nw - g0), 0));
    for (int g0 = 0; g0 < q.nd; g0 += gq) c->h_gblk.push_back(make_int4(i, q.nw + g0, std::min(gq, q.nd - g0), 1));
    for (int k0 = 0; k0 < q.n_probes; k0 += gq) c->h_gblk.push_back(make_int4(i, k0, std::min(gq, q.n_probes - k0), 2));
  }
  c->n_gblk = (int)c->h_gblk.size();
  for (uint32_t w : c->h_wallcount)
    require(w <= WC_BUCKET / 2, "too many wall ghosts in one cell (ghost_layers too large for h/dx)");
  // device memory
  alloc_buf(c, c->b.X);
  alloc_buf(c, c->b.Y);
  alloc_buf(c, c->b.Z);
  alloc_buf(c, c->b.W);
  if (c->scheme == 1) {  // internal energy: the stored state (X) and the sorted state (Y)
    c->b.X.e = dalloc_n<float>(c, c->n_slots);
    c->b.Y.e = dalloc_n<float>(c, c->n_slots);
    HC(hipMemsetAsync(c->b.Y.e, 0, (size_t)c->n_slots * 4, c->st));
  }
  Dev& d = c->d;
  c->d_prm = dalloc_n<InstParams>(c, n_inst);
  // tabulated disk motion (kin_mode 3): WC_KIN_ROWS rows per instance, empty until set
  c->d_kin_tab = dalloc_n<double>(c, (size_t)n_inst * WC_KIN_ROWS * 4);
  for (int i = 0; i < n_inst; ++i) {
    c->hp[i].kin_tab = c->d_kin_tab + (size_t)i * WC_KIN_ROWS * 4;
    c->hp[i].kin_tab_n = 0;
  }
  c->d_clk = dalloc_n<Clock>(c, n_inst);
  d.prm = c->d_prm;
  d.clk = c->d_clk;
  d.n_inst = n_inst;
  d.n_slots = c->n_slots;
  d.n_cells = c->n_cells;
  d.n_ghost = c->n_ghost;
  d.count = dalloc_n<uint32_t>(c, c->n_cells);
  d.start = dalloc_n<uint32_t>(c, c->n_cells + 1);
  c->d_wallcount = dalloc_n<uint32_t>(c, c->n_cells);
  d.wallcount = c->d_wallcount;
  d.bucket_a = dalloc_n<uint32_t>(c, (size_t)c->n_cells * WC_BUCKET);
  d.bucket_b = dalloc_n<uint32_t>(c, (size_t)c->n_cells * WC_BUCKET);
  // per sort tile: bucket entries (two sets) and the static wall-ghost entries
  const size_t n_tiles = ((size_t)c->n_cells + WC_SORT_TILE - 1) / WC_SORT_TILE;
  d.tot_a = dalloc_n<uint32_t>(c, n_tiles);
  d.tot_b = dalloc_n<uint32_t>(c, n_tiles);
  c->d_wall_tot = dalloc_n<uint32_t>(c, n_tiles);
  d.wall_tot = c->d_wall_tot;
  c->n_tiles = n_tiles;
  // (cos, sin) of the ring angles 2 pi k / nd, per instance
  std::vector<double2> ring((size_t)n_inst * WC_MAX_RING, make_double2(0.0, 0.0));
  for (int i = 0; i < n_inst; ++i)
    for (int k = 0; k < c->hp[i].nd; ++k) {
      const double th = 2.0 * M_PI * (double)k / (double)c->hp[i].nd;
      ring[(size_t)i * WC_MAX_RING + k] = make_double2(std::cos(th), std::sin(th));
    }
  double2* ring_cs = dalloc_n<double2>(c, ring.size());
  d.ring_cs = ring_cs;
  HC(hipMemcpyAsync(ring_cs, ring.data(), ring.size() * sizeof(double2), hipMemcpyHostToDevice, c->st));
  d.perm = dalloc_n<uint32_t>(c, c->n_slots);
  d.gslot = dalloc_n<uint32_t>(c, c->n_ghost);
  d.gcell = dalloc_n<uint32_t>(c, c->n_ghost);
  d.gpos = dalloc_n<float2>(c, c->n_ghost);
  c->d_gslot_save = dalloc_n<uint32_t>(c, c->n_ghost);
  uint32_t* wrank = dalloc_n<uint32_t>(c, c->n_ghost);
  d.wrank = wrank;
  int4* gblk = dalloc_n<int4>(c, c->n_gblk);
  d.gblk = gblk;
  d.hist_t = dalloc_n<double>(c, (size_t)n_inst * WC_HIST_CAP);
  d.hist_dt = dalloc_n<double>(c, (size_t)n_inst * WC_HIST_CAP);
  d.hist_p = dalloc_n<float>(c, (size_t)n_inst * WC_HIST_CAP * WC_MAX_PROBES);
  d.diag = dalloc_n<double>(c, (size_t)n_inst * WC_DIAG_CAP * WC_NDIAG);
  d.diag_part = dalloc_n<double>(c, (size_t)n_inst * WC_DIAG_BLOCKS * WC_DIAG_PARTS);
  d.wb_part = dalloc_n<double>(c, (size_t)n_inst * WC_MAX_RING);
  c->d_disk = dalloc_n<double>(c, 3);
  d.var = params[0].kernel_type == 1 ? 2 : 0;
  for (int i = 0; i < n_inst; ++i) {
    if (params[i].beta > 0) d.var |= 1;
    if (params[i].eos_type == 1) d.var |= 4;
  }
  if (c->scheme == 1) d.var |= 8;
  c->audit = !c->batch && params[0].audit != 0;
  d.audit_part = c->audit ? dalloc_n<double>(c, (size_t)wc_pair_blocks(c->n_slots) * 6) : nullptr;
  d.n_vpart = wc_pair_blocks(c->n_slots);
  d.vmax_part = dalloc_n<float>(c, (size_t)d.n_vpart);
  d.xr = dalloc_n<float>(c, (size_t)5 * c->n_slots);
  d.nb_count = dalloc_n<int>(c, c->n_slots);
  d.nb_idsum = dalloc_n<long long>(c, c->n_slots);
  d.n_dt = 0;
  d.dt_step0 = 0;
  d.dt_table = nullptr;
  // axisymmetric instances: each fluid ring's mass per radian r0 m_fluid by
  // particle id, from its set-up radius (kept through set_fluid and load)
  d.mring = nullptr;
  bool any_axisym = false;
  for (int i = 0; i < n_inst; ++i) any_axisym = any_axisym || params[i].axisym;
  if (any_axisym) {
    std::vector<double> mr(c->n_slots, 0.0);
    for (int i = 0; i < n_inst; ++i) {
      const InstParams& q = c->hp[i];
      if (!q.axisym) continue;
      for (int k = 0; k < q.nf; ++k) mr[(size_t)q.id0 + k] = c->geo[i].fy[k] * q.m_fluidd;
    }
    double* dm = dalloc_n<double>(c, c->n_slots);
    HC(hipMemcpyAsync(dm, mr.data(), (size_t)c->n_slots * 8, hipMemcpyHostToDevice, c->st));
    sync(c);  // the host vector goes out of scope
    d.mring = dm;
  }
  HC(hipMemcpyAsync(c->d_prm, c->hp.data(), n_inst * sizeof(InstParams), hipMemcpyHostToDevice, c->st));
  HC(hipMemcpyAsync(c->d_wallcount, c->h_wallcount.data(), (size_t)c->n_cells * 4, hipMemcpyHostToDevice, c->st));
  HC(hipMemcpyAsync(wrank, c->h_wrank.data(), (size_t)c->n_ghost * 4, hipMemcpyHostToDevice, c->st));
  HC(hipMemcpyAsync(gblk, c->h_gblk.data(), (size_t)c->n_gblk * sizeof(int4), hipMemcpyHostToDevice, c->st));
  HC(hipMemsetAsync(d.hist_p, 0, (size_t)n_inst * WC_HIST_CAP * WC_MAX_PROBES * 4, c->st));
  HC(hipMemsetAsync(d.wb_part, 0, (size_t)n_inst * WC_MAX_RING * 8, c->st));
  HC(hipMemsetAsync(d.vmax_part, 0, (size_t)d.n_vpart * 4, c->st));
  {
    std::vector<uint32_t> wt(n_tiles, 0u);
    for (size_t K = 0; K < (size_t)c->n_cells; ++K) wt[K / WC_SORT_TILE] += c->h_wallcount[K];
    HC(hipMemcpyAsync(c->d_wall_tot, wt.data(), n_tiles * 4, hipMemcpyHostToDevice, c->st));
    // set b is re-armed by the first sort; set a is armed with every fill of bucket a
    HC(hipMemcpyAsync(d.tot_b, wt.data(), n_tiles * 4, hipMemcpyHostToDevice, c->st));
    sync(c);  // the host vector goes out of scope
  }
  sync(c);
  c->hist_read.assign(n_inst, 0);
  c->diag_rows.assign(n_inst, 0);
  c->diag_read.assign(n_inst, 0);
  upload_state(c, 0.0, nullptr, nullptr, nullptr, nullptr, nullptr);
  capture(c);
}

void drop_tape_graphs(wcsph_ctx* c);
void release(wcsph_ctx* c) {
  if (c->st) hipStreamSynchronize(c->st);
  drop_graphs(c);
  drop_tape_graphs(c);
  for (void* p : c->blocks) {
    if (c->custom_alloc) c->al.free(p, (void*)c->st, c->al.user);
    else hipFree(p);
  }
  c->blocks.clear();
}

wcsph_status create_impl(const wcsph_params* params, int n_inst, const wcsph_allocator* alloc,
                         void* stream, wcsph_ctx** out, bool batch) {
  if (!out) return WCSPH_E_INVALID;
  *out = nullptr;
  g_create_error.clear();
  if (!params || n_inst < 1 || n_inst > 256) {
    g_create_error = "params must be non-NULL and 1 <= n_inst <= 256";
    return WCSPH_E_INVALID;
  }
  if (!stream) {
    g_create_error = "a non-NULL hipStream_t is required (the step is graph-captured on it)";
    return WCSPH_E_INVALID;
  }
  if (alloc && (!alloc->alloc || !alloc->free)) {
    g_create_error = "allocator needs both alloc and free";
    return WCSPH_E_INVALID;
  }
  try {
    for (int i = 0; i < n_inst; ++i) validate(params[i]);
    for (int i = 1; i < n_inst; ++i)
      require(params[i].diag_every == params[0].diag_every, "batched instances share diag_every");
    if (batch)
      for (int i = 0; i < n_inst; ++i) require(params[i].audit == 0, "the energy audit needs a single-instance context");
    for (int i = 1; i < n_inst; ++i)
      require(params[i].kernel_type == params[0].kernel_type, "batched instances share the kernel");
  } catch (const WcError& e) {
    g_create_error = e.msg;
    return e.st;
  }
  wcsph_ctx* c = new wcsph_ctx();
  c->st = (hipStream_t)stream;
  c->batch = batch;
  if (alloc) {
    c->al = *alloc;
    c->custom_alloc = true;
  }
  try {
    c->scratch = static_cast<uint32_t*>(scratch_address());
    build(c, params, n_inst);
  } catch (const WcError& e) {
    g_create_error = e.msg;
    release(c);
    delete c;
    return e.st;
  }
  *out = c;
  return WCSPH_OK;
}

// Save / restore what the test hooks disturb: sort counters, ghost slots
// and clocks (the state in X itself is left untouched by the hooks).
struct HookGuard {
  wcsph_ctx* c;
  Clock one;                // single-instance contexts: no host allocation
  std::vector<Clock> many;  // batched contexts
  Clock* clk;
  explicit HookGuard(wcsph_ctx* cc) : c(cc), clk(&one) {
    sync(c);
    // scheme 1 after an odd step count: the pending entries are in bucket
    // set b; the hooks' sort reads set a, so refill it from the state
    if (c->scheme == 1 && c->lf_set != 0) {
      rearm(c);
      sync(c);
    }
    if (c->n_inst > 1) {
      many.resize(c->n_inst);
      clk = many.data();
    }
    HC(hipMemcpy(clk, c->d_clk, (size_t)c->n_inst * sizeof(Clock), hipMemcpyDeviceToHost));
    HC(hipMemcpyAsync(c->d_gslot_save, c->d.gslot, (size_t)c->n_ghost * 4, hipMemcpyDeviceToDevice, c->st));
  }
  void restore() {
    HC(hipMemcpyAsync(c->d.gslot, c->d_gslot_save, (size_t)c->n_ghost * 4, hipMemcpyDeviceToDevice, c->st));
    sync(c);
    for (int i = 0; i < c->n_inst; ++i) {
      Clock k = clk[i];
      k.vmax_bits = 0u;
      HC(hipMemcpy(c->d_clk + i, &k, sizeof(Clock), hipMemcpyHostToDevice));
    }
    rearm(c);
    sync(c);
    // the fluid |v| max is recomputed; keep the larger of it and the saved value
    for (int i = 0; i < c->n_inst; ++i) {
      Clock now;
      HC(hipMemcpy(&now, c->d_clk + i, sizeof(Clock), hipMemcpyDeviceToHost));
      now.vmax_bits = std::max(now.vmax_bits, clk[i].vmax_bits);
      HC(hipMemcpy(c->d_clk + i, &now, sizeof(Clock), hipMemcpyHostToDevice));
    }
  }
};

template <class T>
std::vector<T> d2h(wcsph_ctx* c, const T* p, size_t n) {
  std::vector<T> v(n);
  if (n) HC(hipMemcpy(v.data(), p, n * sizeof(T), hipMemcpyDeviceToHost));
  return v;
}

// The neighbour-list export: one cell-list build, ghost pass and pair pass
// of the current state with the export buffer `buf` (per fluid index: the
// count, then WC_NB_CAP ids), copied into the caller's count[nf] and
// nbr[nf][max_per] arrays. No allocation; the caller restores the state.
void check_list_export(wcsph_ctx* ctx, const int* count, const unsigned* nbr, int max_per, int n_fluid) {
  require(!ctx->batch, "single-instance contexts only");
  require(max_per >= 1 && count != nullptr && nbr != nullptr, "count and nbr required");
  if (n_fluid < ctx->hp[0].nf) throw WcError{WCSPH_E_RANGE, "output arrays shorter than the fluid count"};
}
size_t list_export_words(const wcsph_ctx* ctx) { return (size_t)ctx->hp[0].nf * (WC_NB_CAP + 1); }
void list_export(wcsph_ctx* ctx, uint32_t* buf, int* count, unsigned* nbr, int max_per) {
  const size_t nf = (size_t)ctx->hp[0].nf;
  wc_enqueue_export_sort(ctx->d, ctx->b, false, ctx->st);
  if (ctx->scheme == 1) wc_enqueue_export_dens(ctx->d, ctx->b, ctx->st);
  wc_enqueue_export_ghosts(ctx->d, ctx->b, ctx->n_gblk, ctx->st);
  HC(hipMemsetAsync(buf, 0, nf * sizeof(uint32_t), ctx->st));
  Dev dl = ctx->d;
  dl.nb_ids = buf;
  wc_enqueue_export_pair(dl, ctx->b, ctx->st);
  HC(hipGetLastError());
  HC(hipMemcpyAsync(count, buf, nf * sizeof(int), hipMemcpyDeviceToHost, ctx->st));
  const size_t w = (size_t)std::min(max_per, WC_NB_CAP) * sizeof(uint32_t);
  HC(hipMemcpy2DAsync(nbr, (size_t)max_per * sizeof(unsigned), buf + nf, WC_NB_CAP * sizeof(uint32_t), w, nf,
                      hipMemcpyDeviceToHost, ctx->st));
  sync(ctx);
}
bool list_export_over(const wcsph_ctx* ctx, const int* count, int max_per) {
  const int cap = std::min(max_per, WC_NB_CAP);
  for (int k = 0; k < ctx->hp[0].nf; ++k)
    if (count[k] > cap) return true;
  return false;
}

// Device-side checkpoint of the whole evolving state (X buffer, clocks,
// ghost slots); the buckets of the next sort are refilled on restore.
size_t ckpt_size(const wcsph_ctx* c) {
  return (size_t)c->n_slots * 40 + (size_t)c->n_inst * sizeof(Clock) + (size_t)c->n_ghost * 4 + 256;
}
void ckpt_copy(wcsph_ctx* c, char* blob, bool save) {
  const size_t N = c->n_slots;
  size_t off = 0;
  auto mv = [&](void* dev, size_t bytes) {
    if (save) HC(hipMemcpyAsync(blob + off, dev, bytes, hipMemcpyDeviceToDevice, c->st));
    else HC(hipMemcpyAsync(dev, blob + off, bytes, hipMemcpyDeviceToDevice, c->st));
    off += (bytes + 15) & ~size_t(15);
  };
  mv(c->b.X.cell, N * 4);
  mv(c->b.X.id, N * 4);
  mv(c->b.X.pv, N * 16);
  mv(c->b.X.aux, N * 16);
  mv(c->d_clk, c->n_inst * sizeof(Clock));
  mv(c->d.gslot, (size_t)c->n_ghost * 4);
  if (!save) rearm(c);
}

// The tape of steps [tape_steps, steps): one device block for all of them,
// carved into the evaluations' arrays (256-byte aligned), so that a long
// tape costs one allocation.
void alloc_tape(wcsph_ctx* c, int steps) {
  auto& A = c->adj;
  if (A.tape_steps >= steps) return;
  const size_t N = c->n_slots, nf = c->hp[0].nf;
  auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
  const size_t per_eval = 2 * al(N * 4) + 2 * al(N * 16) + al(((size_t)c->n_cells + 1) * 4) +
                          al((size_t)c->n_ghost * 4) + 2 * al(nf * 16);
  char* slab = static_cast<char*>(dalloc(c, per_eval * 2 * (size_t)(steps - A.tape_steps)));
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char* q = slab + off;
    off += al(bytes);
    return q;
  };
  for (int k = A.tape_steps; k < steps; ++k) {
    for (int e = 0; e < 2; ++e) {
      TapeEval t;
      t.cell = reinterpret_cast<uint32_t*>(take(N * 4));
      t.id = reinterpret_cast<uint32_t*>(take(N * 4));
      t.pv = reinterpret_cast<float4*>(take(N * 16));
      t.aux = reinterpret_cast<float4*>(take(N * 16));
      t.start = reinterpret_cast<uint32_t*>(take(((size_t)c->n_cells + 1) * 4));
      t.gslot = reinterpret_cast<uint32_t*>(take((size_t)c->n_ghost * 4));
      (e == 0 ? A.tA : A.tB).push_back(t);
      (e == 0 ? A.pA : A.pB).push_back(reinterpret_cast<double2*>(take(nf * 16)));
      (e == 0 ? A.vA : A.vB).push_back(reinterpret_cast<float4*>(take(nf * 16)));
    }
  }
  A.tape_steps = steps;
}

// A sorted-state buffer that lives in the tape (the batched instance tags of
// the working buffer are kept).
Buf tape_buf(const Buf& work, const TapeEval& t) {
  Buf b = work;
  b.cell = t.cell;
  b.id = t.id;
  b.pv = t.pv;
  b.aux = t.aux;
  return b;
}

// Re-run local steps [0, n) of a segment from its checkpoint with plain
// launches. Each evaluation sorts straight into its tape entry (sorted
// state, cell ranges, ghost slots); the enforcement kernels tape the
// pre-enforcement state. The corrector's pair kernel reads the predictor's
// sorted state from the tape as well.
void replay_taped_step(wcsph_ctx* c, int k) {
  auto& A = c->adj;
  Bufs bt = c->b;
  bt.Y = tape_buf(c->b.Y, A.tA[k]);
  bt.W = tape_buf(c->b.W, A.tB[k]);
  Dev dA = c->d;
  dA.start = A.tA[k].start;
  dA.gslot = A.tA[k].gslot;
  dA.tape_pos = A.pA[k];
  dA.tape_vel = A.vA[k];
  wc_enqueue_eval(dA, bt, c->n_gblk, EV_A, c->st);
  HC(hipGetLastError());
  Dev dB = c->d;
  dB.start = A.tB[k].start;
  dB.gslot = A.tB[k].gslot;
  dB.tape_pos = A.pB[k];
  dB.tape_vel = A.vB[k];
  wc_enqueue_eval(dB, bt, c->n_gblk, EV_B, c->st);
  HC(hipGetLastError());
}
void replay_taped(wcsph_ctx* c, int n) {
  for (int k = 0; k < n; ++k) replay_taped_step(c, k);
}

// The forward's taping of n steps through graphs of WC_TAPE_GRAPH_STEPS
// steps each (the same launches as replay_taped), captured once and kept
// while the step count, the device state handed to the kernels and the
// buffers stay as they were.
#define WC_TAPE_GRAPH_STEPS 10
void drop_tape_graphs(wcsph_ctx* c) {
  auto& A = c->adj;
  for (hipGraphExec_t e : A.tg_exec) hipGraphExecDestroy(e);
  for (hipGraph_t g : A.tg_graph) hipGraphDestroy(g);
  A.tg_exec.clear();
  A.tg_graph.clear();
  A.tg_n = 0;
}
void taped_forward(wcsph_ctx* c, int n) {
  auto& A = c->adj;
  if (A.tg_n != n || std::memcmp(&A.tg_dev, &c->d, sizeof(Dev)) != 0 ||
      std::memcmp(&A.tg_bufs, &c->b, sizeof(Bufs)) != 0) {
    drop_tape_graphs(c);
    for (int k0 = 0; k0 < n; k0 += WC_TAPE_GRAPH_STEPS) {
      hipGraph_t g = nullptr;
      hipGraphExec_t e = nullptr;
      HC(hipStreamBeginCapture(c->st, hipStreamCaptureModeThreadLocal));
      for (int k = k0; k < std::min(n, k0 + WC_TAPE_GRAPH_STEPS); ++k) replay_taped_step(c, k);
      HC(hipStreamEndCapture(c->st, &g));
      A.tg_graph.push_back(g);
      HC(hipGraphInstantiate(&e, g, nullptr, nullptr, 0));
      A.tg_exec.push_back(e);
    }
    A.tg_n = n;
    std::memcpy(&A.tg_dev, &c->d, sizeof(Dev));
    std::memcpy(&A.tg_bufs, &c->b, sizeof(Bufs));
  }
  for (hipGraphExec_t e : A.tg_exec) HC(hipGraphLaunch(e, c->st));
}

}  // namespace

#define API_BEGIN(ctx)                                   \
  if (!(ctx)) return WCSPH_E_STATE;                      \
  if ((ctx)->dead) {                                     \
    (ctx)->err = "context unusable after a HIP error";   \
    return WCSPH_E_STATE;                                \
  }                                                      \
  try {
#define API_END(ctx)                                     \
  }                                                      \
  catch (const WcError& e) {                             \
    (ctx)->err = e.msg;                                  \
    if (e.st == WCSPH_E_HIP) (ctx)->dead = true;         \
    return e.st;                                         \
  }                                                      \
  catch (const std::exception& e) {                      \
    (ctx)->err = e.what();                               \
    return WCSPH_E_INVALID;                              \
  }                                                      \
  return WCSPH_OK;

extern "C" {

wcsph_status wcsph_create(const wcsph_params* p, const wcsph_allocator* alloc, void* stream,
                          wcsph_ctx** out) {
  return create_impl(p, 1, alloc, stream, out, false);
}

wcsph_status wcsph_batch_create(const wcsph_params* params, int n_inst, const wcsph_allocator* alloc,
                                void* stream, wcsph_ctx** out) {
  return create_impl(params, n_inst, alloc, stream, out, true);
}

wcsph_status wcsph_destroy(wcsph_ctx* ctx) {
  if (!ctx) return WCSPH_E_STATE;
  release(ctx);
  delete ctx;
  return WCSPH_OK;
}

const char* wcsph_last_error(const wcsph_ctx* ctx) {
  return ctx ? ctx->err.c_str() : g_create_error.c_str();
}

wcsph_status wcsph_get_info(const wcsph_ctx* ctx, wcsph_info* out) {
  if (!ctx) return WCSPH_E_STATE;
  if (!out) return WCSPH_E_INVALID;
  out->n_inst = ctx->n_inst;
  out->n_fluid = ctx->n_fluid;
  out->n_ghost = ctx->n_ghost;
  out->n_slots = ctx->n_slots;
  out->n_cells = ctx->n_cells;
  out->steps = ctx->steps;
  return WCSPH_OK;
}

wcsph_status wcsph_instance_info(const wcsph_ctx* ctx, int inst, int* n_fluid, int* n_ghost, int* n_cells) {
  if (!ctx) return WCSPH_E_STATE;
  if (inst < 0 || inst >= ctx->n_inst) return WCSPH_E_INVALID;
  const InstParams& q = ctx->hp[inst];
  if (n_fluid) *n_fluid = q.nf;
  if (n_ghost) *n_ghost = q.nw + q.nd;
  if (n_cells) *n_cells = q.ncell;
  return WCSPH_OK;
}

wcsph_status wcsph_set_disk_kinematics(wcsph_ctx* ctx, int inst, int mode, const double* coeffs, int n) {
  API_BEGIN(ctx)
  require(inst >= 0 && inst < ctx->n_inst, "instance out of range");
  require(mode >= 0 && mode <= 3, "mode must be 0, 1, 2 or 3");
  require(coeffs != nullptr, "coefficients required");
  if (mode == 3) {
    require(n >= 1 && n <= WC_KIN_ROWS, "a table of 1 to " + std::to_string(WC_KIN_ROWS) + " rows expected");
    for (int k = 0; k < 4 * n; ++k) require(std::isfinite(coeffs[k]), "the table must be finite");
    for (int k = 1; k < n; ++k) require(coeffs[4 * k] > coeffs[4 * (k - 1)], "table times must increase");
  } else {
    require(n == 3, "three coefficients expected");
    require(coeffs[0] >= 0 && coeffs[1] > 0 && coeffs[2] >= 0, "coefficients must be non-negative, t_ramp > 0");
  }
  if (mode == 2 && ctx->hp[inst].nd > 0)
    require(ctx->hp[inst].disk_mass > 0 && std::isfinite(ctx->hp[inst].disk_mass),
            "a two-way coupled disk needs disk_mass > 0");
  sync(ctx);
  InstParams& q = ctx->hp[inst];
  q.kin_mode = mode;
  ctx->pin[inst].kin_mode = mode;
  if (mode == 3) {
    HC(hipMemcpy(const_cast<double*>(q.kin_tab), coeffs, (size_t)n * 4 * sizeof(double), hipMemcpyHostToDevice));
    q.kin_tab_n = n;
  } else {
    q.kin_v0 = coeffs[0];
    q.kin_t_ramp = coeffs[1];
    q.kin_coef = coeffs[2];
    ctx->pin[inst].kin_v0 = coeffs[0];
    ctx->pin[inst].kin_t_ramp = coeffs[1];
    ctx->pin[inst].kin_coef = coeffs[2];
  }
  HC(hipMemcpyAsync(ctx->d_prm + inst, &q, sizeof(InstParams), hipMemcpyHostToDevice, ctx->st));
  // the new law starts from the newest state: a coupled disk is released
  // (mode 2 couples again at its next step at or after t_ramp)
  const int zero = 0;
  HC(hipMemcpyAsync(reinterpret_cast<char*>(ctx->d_clk + inst) + offsetof(Clock, coupled), &zero, sizeof zero,
                    hipMemcpyHostToDevice, ctx->st));
  // the ring of the newest state was placed with the old law: place it again
  rearm(ctx);
  sync(ctx);
  // the step graph launches the disk update only when some disk is coupled
  capture(ctx);
  API_END(ctx)
}

wcsph_status wcsph_set_dt_table(wcsph_ctx* ctx, const double* dt, int n) {
  API_BEGIN(ctx)
  require(n >= 0 && (n == 0 || dt != nullptr), "dt table invalid");
  for (int k = 0; k < n; ++k) require(dt[k] > 0 && std::isfinite(dt[k]), "dt entries must be positive");
  sync(ctx);
  if ((size_t)n > ctx->d_dt_cap) {
    ctx->d_dt = dalloc_n<double>(ctx, n);
    ctx->d_dt_cap = n;
  }
  if (n) HC(hipMemcpy(ctx->d_dt, dt, (size_t)n * 8, hipMemcpyHostToDevice));
  ctx->d.dt_table = ctx->d_dt;
  ctx->d.n_dt = n;
  ctx->d.dt_step0 = ctx->steps;
  capture(ctx);
  API_END(ctx)
}

wcsph_status wcsph_step(wcsph_ctx* ctx, int n_steps) {
  API_BEGIN(ctx)
  require(n_steps >= 0, "n_steps must be >= 0");
  const int de = ctx->diag_every, K = ctx->steps_k;
  int n = n_steps;
  while (n > 0) {
    const bool b_set = ctx->scheme == 1 && ctx->lf_set != 0;
    if (n >= K && (de <= 0 || ctx->steps % de == 0)) {
      HC(hipGraphLaunch(b_set ? ctx->gexec_k1 : ctx->gexec_k, ctx->st));
      ctx->steps += K;
      n -= K;
      if (ctx->scheme == 1) ctx->lf_set ^= (K & 1);
      if (de > 0)
        for (int i = 0; i < ctx->n_inst; ++i) ctx->diag_rows[i]++;
      continue;
    }
    HC(hipGraphLaunch(b_set ? ctx->gexec1 : ctx->gexec, ctx->st));
    ctx->steps++;
    if (ctx->scheme == 1) ctx->lf_set ^= 1;
    --n;
    if (de > 0 && ctx->steps % de == 0) {
      wc_enqueue_diag(ctx->d, ctx->b, true, ctx->st);
      HC(hipGetLastError());
      for (int i = 0; i < ctx->n_inst; ++i) ctx->diag_rows[i]++;
    }
  }
  API_END(ctx)
}

wcsph_status wcsph_batch_step(wcsph_ctx* ctx, int n_steps) {
  if (ctx && !ctx->dead && !ctx->batch) {
    ctx->err = "wcsph_batch_step needs a context from wcsph_batch_create";
    return WCSPH_E_INVALID;
  }
  return wcsph_step(ctx, n_steps);
}

wcsph_status wcsph_synchronize(wcsph_ctx* ctx) {
  API_BEGIN(ctx)
  sync(ctx);
  API_END(ctx)
}

wcsph_status wcsph_read_probes(wcsph_ctx* ctx, int inst, double* t, double* dt, float* p, int max_rows,
                               int* rows_out) {
  API_BEGIN(ctx)
  require(inst >= 0 && inst < ctx->n_inst, "instance out of range");
  require(max_rows >= 0 && rows_out != nullptr, "rows_out required");
  sync(ctx);
  long long& rd = ctx->hist_read[inst];
  if (ctx->steps - rd > WC_HIST_CAP) rd = ctx->steps - WC_HIST_CAP;
  const long long rows = std::min<long long>(ctx->steps - rd, max_rows);
  const int np = ctx->hp[inst].n_probes;
  const size_t base = (size_t)inst * WC_HIST_CAP;
  // the rows are at most two contiguous runs of the ring
  std::vector<float> rowbuf;
  for (long long r = 0; r < rows;) {
    const size_t k0 = (size_t)((rd + r) % WC_HIST_CAP);
    const long long run = std::min<long long>(rows - r, (long long)(WC_HIST_CAP - k0));
    if (t) HC(hipMemcpy(t + r, ctx->d.hist_t + base + k0, (size_t)run * 8, hipMemcpyDeviceToHost));
    if (dt) HC(hipMemcpy(dt + r, ctx->d.hist_dt + base + k0, (size_t)run * 8, hipMemcpyDeviceToHost));
    if (p && np) {
      rowbuf.resize((size_t)run * WC_MAX_PROBES);
      HC(hipMemcpy(rowbuf.data(), ctx->d.hist_p + (base + k0) * WC_MAX_PROBES, rowbuf.size() * 4,
                   hipMemcpyDeviceToHost));
      for (long long q = 0; q < run; ++q)
        std::copy(rowbuf.begin() + q * WC_MAX_PROBES, rowbuf.begin() + q * WC_MAX_PROBES + np, p + (r + q) * np);
    }
    r += run;
  }
  rd += rows;
  *rows_out = (int)rows;
  if (state_invalid(ctx, inst)) return WCSPH_E_UNSTABLE;
  API_END(ctx)
}

wcsph_status wcsph_read_diagnostics(wcsph_ctx* ctx, int inst, wcsph_diag* out, int max, int* n_out) {
  API_BEGIN(ctx)
  require(inst >= 0 && inst < ctx->n_inst, "instance out of range");
  require(max >= 0 && n_out != nullptr, "n_out required");
  sync(ctx);
  long long& rd = ctx->diag_read[inst];
  if (ctx->diag_rows[inst] - rd > WC_DIAG_CAP) rd = ctx->diag_rows[inst] - WC_DIAG_CAP;
  const long long rows = std::min<long long>(ctx->diag_rows[inst] - rd, max);
  // the rows are at most two contiguous runs of the ring
  std::vector<double> all((size_t)rows * WC_NDIAG);
  for (long long r = 0; r < rows;) {
    const size_t k0 = (size_t)((rd + r) % WC_DIAG_CAP);
    const long long run = std::min<long long>(rows - r, (long long)(WC_DIAG_CAP - k0));
    HC(hipMemcpy(all.data() + (size_t)r * WC_NDIAG, ctx->d.diag + ((size_t)inst * WC_DIAG_CAP + k0) * WC_NDIAG,
                 (size_t)run * WC_NDIAG * sizeof(double), hipMemcpyDeviceToHost));
    r += run;
  }
  for (long long r = 0; r < rows; ++r) {
    const double* v = all.data() + (size_t)r * WC_NDIAG;
    wcsph_diag& o = out[r];
    o.t = v[0];
    o.dt = v[1];
    o.vmax = v[2];
    o.mass = v[3];
    o.mom[0] = v[4];
    o.mom[1] = v[5];
    o.ke = v[6];
    o.e_el = v[7];
    o.e_pot = v[8];
    o.e_disk = v[9];
    o.w_boundary = v[10];
    o.step = (long long)v[11];
    o.n_clamp = (long long)v[12];
    o.n_cav = (long long)v[13];
    o.n_enforce = (long long)v[14];
    o.d_av = v[15];
    o.d_visc = v[16];
    o.w_delta = v[17];
    o.w_ghost = v[18];
    o.w_enforce = v[19];
    o.w_clamp = v[20];
    o.e_th = v[21];
  }
  rd += rows;
  *n_out = (int)rows;
  if (state_invalid(ctx, inst)) return WCSPH_E_UNSTABLE;
  API_END(ctx)
}

wcsph_status wcsph_get_fluid(wcsph_ctx* ctx, int inst, double* t, double* x, double* y, double* vx, double* vy,
                             double* rho, int n) {
  API_BEGIN(ctx)
  require(inst >= 0 && inst < ctx->n_inst, "instance out of range");
  const InstParams& q = ctx->hp[inst];
  if (n < q.nf) throw WcError{WCSPH_E_RANGE, "output arrays shorter than the fluid count"};
  sync(ctx);
  const size_t N = ctx->n_slots;
  auto cell = d2h(ctx, ctx->b.X.cell, N);
  auto id = d2h(ctx, ctx->b.X.id, N);
  auto pv = d2h(ctx, ctx->b.X.pv, N);
  auto aux = d2h(ctx, ctx->b.X.aux, N);
  for (size_t s = 0; s < N; ++s) {
    const int k = (int)id[s] - q.id0;
    if (k < 0 || k >= q.nf) continue;
    double xx, yy;
    decode(q, cell[s], pv[s].x, pv[s].y, xx, yy);
    if (x) x[k] = xx;
    if (y) y[k] = yy;
    if (vx) vx[k] = pv[s].z;
    if (vy) vy[k] = pv[s].w;
    if (rho) rho[k] = aux[s].x;
  }
  if (t) {
    Clock k;
    HC(hipMemcpy(&k, ctx->d_clk + inst, sizeof k, hipMemcpyDeviceToHost));
    *t = k.t_next;
  }
  if (state_invalid(ctx, inst)) return WCSPH_E_UNSTABLE;
  API_END(ctx)
}

wcsph_status wcsph_get_internal_energy(wcsph_ctx* ctx, int inst, double* e, int n) {
  API_BEGIN(ctx)
  require(inst >= 0 && inst < ctx->n_inst, "instance out of range");
  require(e != nullptr, "e required");
  const InstParams& q = ctx->hp[inst];
  if (n < q.nf) throw WcError{WCSPH_E_RANGE, "output array shorter than the fluid count"};
  sync(ctx);
  for (int k = 0; k < q.nf; ++k) e[k] = 0.0;
  if (ctx->b.X.e) {
    const size_t N = ctx->n_slots;
    auto id = d2h(ctx, ctx->b.X.id, N);
    auto ev = d2h(ctx, ctx->b.X.e, N);
    for (size_t s = 0; s < N; ++s) {
      const int k = (int)id[s] - q.id0;
      if (k >= 0 && k < q.nf) e[k] = ev[s];
    }
  }
  if (state_invalid(ctx, inst)) return WCSPH_E_UNSTABLE;
  API_END(ctx)
}

wcsph_status wcsph_get_disk(wcsph_ctx* ctx, int inst, double* x, double* v, double* a) {
  API_BEGIN(ctx)
  require(inst >= 0 && inst < ctx->n_inst, "instance out of range");
  wc_enqueue_disk_query(ctx->d, inst, ctx->d_disk, ctx->st);
  HC(hipGetLastError());
  double o[3];
  HC(hipMemcpyAsync(o, ctx->d_disk, sizeof o, hipMemcpyDeviceToHost, ctx->st));
  sync(ctx);
  if (x) *x = o[0];
  if (v) *v = o[1];
  if (a) *a = o[2];
  if (state_invalid(ctx, inst)) return WCSPH_E_UNSTABLE;
  API_END(ctx)
}

wcsph_status wcsph_set_fluid(wcsph_ctx* ctx, double t, const double* x, const double* y, const double* vx,
                             const double* vy, const double* rho, int n) {
  API_BEGIN(ctx)
  require(ctx->n_inst == 1, "set_fluid needs a single-instance context");
  require(x && y && vx && vy && rho, "all arrays required");
  require(n == ctx->hp[0].nf, "n must equal the fluid count");
  for (int k = 0; k < n; ++k)
    require(std::isfinite(x[k]) && std::isfinite(y[k]) && std::isfinite(vx[k]) && std::isfinite(vy[k]) &&
                rho[k] > 0,
            "non-finite or non-positive input");
  sync(ctx);
  upload_state(ctx, t, x, y, vx, vy, rho);
  if (ctx->d.n_dt > 0 && ctx->d.dt_step0 != 0) {
    ctx->d.dt_step0 = 0;
    capture(ctx);
  }
  API_END(ctx)
}

namespace {
struct BlobHeader {
  char magic[8];
  long long n_inst, n_slots, n_cells, n_ghost, steps, batch, n_audit;
};
size_t audit_bytes(const wcsph_ctx* c) { return c->d.audit_part ? (size_t)c->d.n_vpart * 6 * sizeof(double) : 0; }
// scheme 1: the internal energy per slot, after everything else
size_t energy_bytes(const wcsph_ctx* c) { return c->b.X.e ? (size_t)c->n_slots * 4 : 0; }
}  // namespace

wcsph_status wcsph_save_state(wcsph_ctx* ctx, void* buf, size_t cap, size_t* need) {
  API_BEGIN(ctx)
  const size_t N = ctx->n_slots;
  const size_t sz = sizeof(BlobHeader) + ctx->n_inst * sizeof(Clock) + N * (4 + 4 + 16 + 16 + 2) +
                    (size_t)ctx->n_ghost * 4 + audit_bytes(ctx) + energy_bytes(ctx);
  if (need) *need = sz;
  if (!buf) return WCSPH_OK;
  if (cap < sz) throw WcError{WCSPH_E_RANGE, "buffer too small for the state"};
  sync(ctx);
  char* o = static_cast<char*>(buf);
  BlobHeader h;
  std::memset(&h, 0, sizeof h);
  std::memcpy(h.magic, "WCSPHST4", 8);
  h.n_inst = ctx->n_inst;
  h.n_slots = N;
  h.n_cells = ctx->n_cells;
  h.n_ghost = ctx->n_ghost;
  h.steps = ctx->steps;
  h.batch = ctx->batch;
  h.n_audit = (long long)audit_bytes(ctx);
  std::memcpy(o, &h, sizeof h);
  o += sizeof h;
  auto put = [&](const void* dev, size_t bytes) {
    HC(hipMemcpy(o, dev, bytes, hipMemcpyDeviceToHost));
    o += bytes;
  };
  put(ctx->d_clk, ctx->n_inst * sizeof(Clock));
  put(ctx->b.X.cell, N * 4);
  put(ctx->b.X.id, N * 4);
  put(ctx->b.X.pv, N * 16);
  put(ctx->b.X.aux, N * 16);
  if (ctx->batch) put(ctx->b.X.inst, N * 2);
  else {
    std::memset(o, 0, N * 2);
    o += N * 2;
  }
  put(ctx->d.gslot, (size_t)ctx->n_ghost * 4);
  if (ctx->d.audit_part) put(ctx->d.audit_part, audit_bytes(ctx));
  if (ctx->b.X.e) put(ctx->b.X.e, energy_bytes(ctx));
  API_END(ctx)
}

wcsph_status wcsph_load_state(wcsph_ctx* ctx, const void* buf, size_t n) {
  API_BEGIN(ctx)
  require(buf != nullptr && n >= sizeof(BlobHeader), "buffer too small");
  BlobHeader h;
  std::memcpy(&h, buf, sizeof h);
  require(std::memcmp(h.magic, "WCSPHST4", 8) == 0, "not a state blob");
  require(h.n_inst == ctx->n_inst && h.n_slots == ctx->n_slots && h.n_cells == ctx->n_cells &&
              h.n_ghost == ctx->n_ghost && h.batch == (long long)ctx->batch &&
              h.n_audit == (long long)audit_bytes(ctx),
          "state blob does not match this context");
  const size_t N = ctx->n_slots;
  const size_t sz = sizeof(BlobHeader) + ctx->n_inst * sizeof(Clock) + N * (4 + 4 + 16 + 16 + 2) +
                    (size_t)ctx->n_ghost * 4 + audit_bytes(ctx) + energy_bytes(ctx);
  require(n >= sz, "state blob truncated");
  sync(ctx);
  const char* o = static_cast<const char*>(buf) + sizeof h;
  auto get = [&](void* dev, size_t bytes) {
    HC(hipMemcpy(dev, o, bytes, hipMemcpyHostToDevice));
    o += bytes;
  };
  get(ctx->d_clk, ctx->n_inst * sizeof(Clock));
  get(ctx->b.X.cell, N * 4);
  get(ctx->b.X.id, N * 4);
  get(ctx->b.X.pv, N * 16);
  get(ctx->b.X.aux, N * 16);
  if (ctx->batch) get(ctx->b.X.inst, N * 2);
  else o += N * 2;
  get(ctx->d.gslot, (size_t)ctx->n_ghost * 4);
  if (ctx->d.audit_part) get(ctx->d.audit_part, audit_bytes(ctx));
  if (ctx->b.X.e) get(ctx->b.X.e, energy_bytes(ctx));
  rearm(ctx);
  sync(ctx);
  ctx->steps = h.steps;
  std::vector<Clock> clk(ctx->n_inst);
  HC(hipMemcpy(clk.data(), ctx->d_clk, clk.size() * sizeof(Clock), hipMemcpyDeviceToHost));
  for (int i = 0; i < ctx->n_inst; ++i) {
    ctx->hist_read[i] = ctx->steps;
    ctx->diag_rows[i] = clk[i].diag_row;
    ctx->diag_read[i] = ctx->diag_rows[i];
  }
  API_END(ctx)
}

wcsph_status wcsph_export_cells(wcsph_ctx* ctx, unsigned* keys, unsigned* ids_pre, double* x, double* y,
                                unsigned* perm, unsigned* ids_post, unsigned* cell_start, size_t cap_slots,
                                size_t cap_cells) {
  API_BEGIN(ctx)
  require(!ctx->batch, "single-instance contexts only");
  if (cap_slots < (size_t)ctx->n_slots || cap_cells < (size_t)ctx->n_cells + 1)
    throw WcError{WCSPH_E_RANGE, "output arrays too small"};
  HookGuard guard(ctx);
  wc_enqueue_export_sort(ctx->d, ctx->b, false, ctx->st);
  HC(hipGetLastError());
  sync(ctx);
  const size_t N = ctx->n_slots;
  auto cell = d2h(ctx, ctx->b.X.cell, N);
  auto pv = d2h(ctx, ctx->b.X.pv, N);
  auto idp = d2h(ctx, ctx->b.X.id, N);
  auto pm = d2h(ctx, ctx->d.perm, N);
  auto idq = d2h(ctx, ctx->b.Y.id, N);
  auto cs = d2h(ctx, ctx->d.start, (size_t)ctx->n_cells + 1);
  for (size_t s = 0; s < N; ++s) {
    if (keys) keys[s] = cell[s];
    if (ids_pre) ids_pre[s] = idp[s];
    double xx, yy;
    decode(ctx->hp[0], cell[s], pv[s].x, pv[s].y, xx, yy);
    if (x) x[s] = xx;
    if (y) y[s] = yy;
    if (perm) perm[s] = pm[s];
    if (ids_post) ids_post[s] = idq[s];
  }
  if (cell_start) std::copy(cs.begin(), cs.end(), cell_start);
  guard.restore();
  API_END(ctx)
}

wcsph_status wcsph_export_rates(wcsph_ctx* ctx, float* drho, float* ax, float* ay, float* Vx, float* Vy,
                                float* gp, float* grho, float* gvx, float* gvy, int n_fluid, int n_ghost) {
  API_BEGIN(ctx)
  require(!ctx->batch, "single-instance contexts only");
  const InstParams& q = ctx->hp[0];
  if (n_fluid < q.nf || n_ghost < q.nw + q.nd) throw WcError{WCSPH_E_RANGE, "output arrays too small"};
  HookGuard guard(ctx);
  wc_enqueue_export_sort(ctx->d, ctx->b, false, ctx->st);
  if (ctx->scheme == 1) wc_enqueue_export_dens(ctx->d, ctx->b, ctx->st);
  wc_enqueue_export_ghosts(ctx->d, ctx->b, ctx->n_gblk, ctx->st);
  wc_enqueue_export_pair(ctx->d, ctx->b, ctx->st);
  HC(hipGetLastError());
  sync(ctx);
  const size_t N = ctx->n_slots;
  auto xr = d2h(ctx, ctx->d.xr, 5 * N);
  auto id = d2h(ctx, ctx->b.Y.id, N);
  auto pv = d2h(ctx, ctx->b.Y.pv, N);
  auto aux = d2h(ctx, ctx->b.Y.aux, N);
  for (size_t s = 0; s < N; ++s) {
    const int k = (int)id[s] - q.id0;
    if (k >= 0 && k < q.nf) {
      if (drho) drho[k] = xr[s];
      if (ax) ax[k] = xr[N + s];
      if (ay) ay[k] = xr[2 * N + s];
      if (Vx) Vx[k] = xr[3 * N + s];
      if (Vy) Vy[k] = xr[4 * N + s];
    } else if (k >= q.nf && k < q.nf + q.nw + q.nd) {
      const int g = k - q.nf;
      if (gp) gp[g] = aux[s].y * aux[s].x * aux[s].x;
      if (grho) grho[g] = aux[s].x;
      if (gvx) gvx[g] = pv[s].z;
      if (gvy) gvy[g] = pv[s].w;
    }
  }
  guard.restore();
  API_END(ctx)
}

wcsph_status wcsph_export_density(wcsph_ctx* ctx, float* rho, float* p, int n_fluid) {
  API_BEGIN(ctx)
  require(!ctx->batch, "single-instance contexts only");
  const InstParams& q = ctx->hp[0];
  if (n_fluid < q.nf) throw WcError{WCSPH_E_RANGE, "output arrays too small"};
  HookGuard guard(ctx);
  wc_enqueue_export_sort(ctx->d, ctx->b, false, ctx->st);
  if (ctx->scheme == 1) wc_enqueue_export_dens(ctx->d, ctx->b, ctx->st);
  HC(hipGetLastError());
  sync(ctx);
  const size_t N = ctx->n_slots;
  auto id = d2h(ctx, ctx->b.Y.id, N);
  auto aux = d2h(ctx, ctx->b.Y.aux, N);
  for (size_t s = 0; s < N; ++s) {
    const int k = (int)id[s] - q.id0;
    if (k < 0 || k >= q.nf) continue;
    if (rho) rho[k] = aux[s].x;
    if (p) p[k] = aux[s].y * aux[s].x * aux[s].x;
  }
  guard.restore();
  API_END(ctx)
}

wcsph_status wcsph_export_neighbours(wcsph_ctx* ctx, unsigned* ids, int* count, long long* idsum, double* x,
                                     double* y, size_t cap_slots) {
  API_BEGIN(ctx)
  require(!ctx->batch, "single-instance contexts only");
  if (cap_slots < (size_t)ctx->n_slots) throw WcError{WCSPH_E_RANGE, "output arrays too small"};
  HookGuard guard(ctx);
  wc_enqueue_export_sort(ctx->d, ctx->b, false, ctx->st);
  wc_enqueue_neigh(ctx->d, ctx->b, ctx->st);
  HC(hipGetLastError());
  sync(ctx);
  const size_t N = ctx->n_slots;
  auto id = d2h(ctx, ctx->b.Y.id, N);
  auto cell = d2h(ctx, ctx->b.Y.cell, N);
  auto pv = d2h(ctx, ctx->b.Y.pv, N);
  auto nc = d2h(ctx, ctx->d.nb_count, N);
  auto ns = d2h(ctx, ctx->d.nb_idsum, N);
  for (size_t s = 0; s < N; ++s) {
    if (ids) ids[s] = id[s];
    if (count) count[s] = nc[s];
    if (idsum) idsum[s] = ns[s];
    double xx, yy;
    decode(ctx->hp[0], cell[s], pv[s].x, pv[s].y, xx, yy);
    if (x) x[s] = xx;
    if (y) y[s] = yy;
  }
  guard.restore();
  API_END(ctx)
}

wcsph_status wcsph_export_neighbour_lists(wcsph_ctx* ctx, int* count, unsigned* nbr, int max_per, int n_fluid) {
  API_BEGIN(ctx)
  check_list_export(ctx, count, nbr, max_per, n_fluid);
  if (!ctx->nb_ids) ctx->nb_ids = dalloc_n<uint32_t>(ctx, list_export_words(ctx));
  HookGuard guard(ctx);
  list_export(ctx, ctx->nb_ids, count, nbr, max_per);
  guard.restore();
  if (list_export_over(ctx, count, max_per)) throw WcError{WCSPH_E_RANGE, "a particle has more neighbours than the list holds"};
  API_END(ctx)
}

wcsph_status wcsph_export_neighbour_lists_noalloc(wcsph_ctx* ctx, int* count, unsigned* nbr, int max_per,
                                                  int n_fluid) {
  API_BEGIN(ctx)
  check_list_export(ctx, count, nbr, max_per, n_fluid);
  if (!ctx->scratch) throw WcError{WCSPH_E_STATE, "no scratch array on this context's device"};
  if (list_export_words(ctx) > WC_SCRATCH_WORDS)
    throw WcError{WCSPH_E_RANGE, "the scratch array holds the lists of at most " +
                                     std::to_string(WC_SCRATCH_WORDS / (WC_NB_CAP + 1)) + " fluid particles"};
  HookGuard guard(ctx);  // single instance: no host allocation
  list_export(ctx, ctx->scratch, count, nbr, max_per);
  guard.restore();
  if (list_export_over(ctx, count, max_per)) throw WcError{WCSPH_E_RANGE, "a particle has more neighbours than the list holds"};
  API_END(ctx)
}

wcsph_status wcsph_time_pair_kernel(wcsph_ctx* ctx, int reps, float* avg_ms) {
  API_BEGIN(ctx)
  require(reps >= 1 && reps <= 1000 && avg_ms != nullptr, "reps must lie in [1, 1000]");
  require(ctx->scheme == 0, "the timing hook times the predictor pass of scheme 0");
  HookGuard guard(ctx);
  wc_enqueue_export_sort(ctx->d, ctx->b, ctx->batch, ctx->st);
  if (!ctx->batch) wc_enqueue_export_ghosts(ctx->d, ctx->b, ctx->n_gblk, ctx->st);
  HC(hipGetLastError());
  // back-to-back launches between two events; every launch does the full
  // work of the step's kernel (its bucket fills pile up past the bucket
  // capacity and are flagged, the flag is reset with the rest of the state)
  hipEvent_t e0, e1;
  HC(hipEventCreate(&e0));
  HC(hipEventCreate(&e1));
  HC(hipEventRecord(e0, ctx->st));
  for (int r = 0; r < reps; ++r) wc_enqueue_pair_a(ctx->d, ctx->b, ctx->batch, ctx->st);
  HC(hipEventRecord(e1, ctx->st));
  HC(hipGetLastError());
  HC(hipEventSynchronize(e1));
  float ms = 0;
  HC(hipEventElapsedTime(&ms, e0, e1));
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  *avg_ms = ms / reps;
  guard.restore();
  API_END(ctx)
}

wcsph_status wcsph_set_coefficients(wcsph_ctx* ctx, int inst, double alpha, double delta, double c0) {
  API_BEGIN(ctx)
  require(inst >= 0 && inst < ctx->n_inst, "instance out of range");
  require(alpha >= 0 && delta >= 0 && c0 > 0 && std::isfinite(alpha + delta + c0), "invalid coefficients");
  wcsph_params p = ctx->pin[inst];
  p.alpha = alpha;
  p.delta = delta;
  p.c0 = c0;
  InstParams q = derive(p);
  InstParams& o = ctx->hp[inst];
  // keep layout and geometry, take the re-derived scheme constants
  q.ncx = o.ncx; q.ncy = o.ncy; q.cell_off = o.cell_off; q.ncell = o.ncell;
  q.id0 = o.id0; q.nf = o.nf; q.nw = o.nw; q.nd = o.nd; q.gmap0 = o.gmap0;
  q.n_probes = o.n_probes;
  for (int k = 0; k < WC_MAX_PROBES; ++k) {
    q.probe_cell[k] = o.probe_cell[k];
    q.probe_ox[k] = o.probe_ox[k];
    q.probe_oy[k] = o.probe_oy[k];
  }
  q.kin_mode = o.kin_mode; q.kin_v0 = o.kin_v0; q.kin_t_ramp = o.kin_t_ramp; q.kin_coef = o.kin_coef;
  q.kin_tab = o.kin_tab; q.kin_tab_n = o.kin_tab_n;
  o = q;
  ctx->pin[inst] = p;
  sync(ctx);
  HC(hipMemcpy(ctx->d_prm + inst, &o, sizeof(InstParams), hipMemcpyHostToDevice));
  API_END(ctx)
}

wcsph_status wcsph_adj_forward(wcsph_ctx* ctx, int n_steps, int ckpt_every, double* J) {
  API_BEGIN(ctx)
  require(!ctx->batch && ctx->n_inst == 1, "the reverse sweep needs a single-instance context");
  require(ctx->pin[0].ghost_rho_mode == 0, "the reverse sweep supports the linear ghost density only");
  require(ctx->pin[0].init_mode == 0, "the reverse sweep needs the rest initial state");
  require((ctx->hp[0].kin_mode != 2 && ctx->hp[0].kin_mode != 3) || ctx->hp[0].nd == 0,
          "the reverse sweep needs a closed-form prescribed disk motion (kin_mode 0 or 1)");
  require(ctx->pin[0].beta == 0, "the reverse sweep supports the linear artificial viscosity only (beta = 0)");
  require(ctx->pin[0].eos_type == 0, "the reverse sweep supports the Tait EOS only");
  require(ctx->pin[0].kernel_type == 0, "the reverse sweep supports the Wendland C2 kernel only");
  require(ctx->scheme == 0, "the reverse sweep supports scheme 0 only");
  require(ctx->pin[0].axisym == 0, "the reverse sweep supports the planar form only");
  require(n_steps >= 1 && ckpt_every >= 1, "n_steps and ckpt_every must be >= 1");
  require(n_steps <= WC_HIST_CAP, "n_steps beyond the probe history's capacity");
  const long long k0 = ctx->steps - ctx->d.dt_step0;
  require(ctx->d.n_dt > 0 && k0 >= 0 && k0 + n_steps <= ctx->d.n_dt,
          "a fixed dt table covering the run is required (wcsph_set_dt_table)");
  auto& A = ctx->adj;
  A.fwd_done = false;
  A.n_steps = n_steps;
  A.ckpt = std::min(ckpt_every, n_steps);
  A.n_seg = (n_steps + A.ckpt - 1) / A.ckpt;
  // one segment: the forward itself writes the whole tape (the same kernels
  // as the step graph, launched one by one with the tape's buffers), and the
  // backward replays nothing. (With the energy audit the step graph's
  // corrector also sums the audit terms, so that run keeps the graph.)
  A.taped = A.n_seg == 1 && !ctx->audit;
  A.step0 = ctx->steps;
  std::vector<double> tab(ctx->d.n_dt);
  sync(ctx);
  HC(hipMemcpy(tab.data(), ctx->d_dt, tab.size() * 8, hipMemcpyDeviceToHost));
  Clock ck;
  HC(hipMemcpy(&ck, ctx->d_clk, sizeof ck, hipMemcpyDeviceToHost));
  A.t.assign(n_steps, 0.0);
  A.dt.assign(n_steps, 0.0);
  double t = ck.t_next;
  for (int k = 0; k < n_steps; ++k) {
    A.t[k] = t;
    A.dt[k] = tab[k0 + k];
    t = t + A.dt[k];
  }
  A.ckpt_bytes = ckpt_size(ctx);
  while ((int)A.ckpt_dev.size() < A.n_seg + 1) A.ckpt_dev.push_back(static_cast<char*>(dalloc(ctx, A.ckpt_bytes)));
  ctx->hist_read[0] = ctx->steps;
  if (A.taped) {
    alloc_tape(ctx, n_steps);
    ckpt_copy(ctx, A.ckpt_dev[0], true);
    taped_forward(ctx, n_steps);
    ctx->steps += n_steps;
  } else {
    for (int g = 0; g < A.n_seg; ++g) {
      ckpt_copy(ctx, A.ckpt_dev[g], true);
      const int n = std::min(A.ckpt, n_steps - g * A.ckpt);
      for (int k = 0; k < n; ++k) HC(hipGraphLaunch(ctx->gexec, ctx->st));
      ctx->steps += n;
    }
  }
  ckpt_copy(ctx, A.ckpt_dev[A.n_seg], true);
  // J = sum_n sum_k p_k^n dt_n (probe rows of this run)
  sync(ctx);
  const int np = ctx->hp[0].n_probes;
  // (the run's rows in one copy, two where the history ring wraps)
  std::vector<float> pr((size_t)n_steps * WC_MAX_PROBES);
  const size_t r0 = (size_t)(A.step0 % WC_HIST_CAP), n1 = std::min((size_t)n_steps, (size_t)WC_HIST_CAP - r0);
  HC(hipMemcpy(pr.data(), ctx->d.hist_p + r0 * WC_MAX_PROBES, n1 * WC_MAX_PROBES * sizeof(float),
               hipMemcpyDeviceToHost));
  if (n1 < (size_t)n_steps)
    HC(hipMemcpy(pr.data() + n1 * WC_MAX_PROBES, ctx->d.hist_p, ((size_t)n_steps - n1) * WC_MAX_PROBES * sizeof(float),
                 hipMemcpyDeviceToHost));
  double Jv = 0.0;
  for (int k = 0; k < n_steps; ++k)
    for (int j = 0; j < np; ++j) Jv += (double)pr[(size_t)k * WC_MAX_PROBES + j] * A.dt[k];
  ctx->hist_read[0] = ctx->steps;
  A.J = Jv;
  if (J) *J = Jv;
  // a run that left the valid state gives no J to differentiate
  if (state_invalid(ctx, 0)) return WCSPH_E_UNSTABLE;
  A.fwd_done = true;
  API_END(ctx)
}

wcsph_status wcsph_adj_backward(wcsph_ctx* ctx, double dJ, double* grad) {
  API_BEGIN(ctx)
  auto& A = ctx->adj;
  if (!A.fwd_done) throw WcError{WCSPH_E_STATE, "wcsph_adj_forward must run first"};
  require(grad != nullptr, "grad[3] required");
  const InstParams& q = ctx->hp[0];
  const int nf = q.nf;
  alloc_tape(ctx, A.ckpt);
  if (!A.L0) {
    A.L0 = dalloc_n<float>(ctx, (size_t)5 * nf);
    A.L1 = dalloc_n<float>(ctx, (size_t)5 * nf);
    A.Ls = dalloc_n<float>(ctx, (size_t)5 * nf);
    A.a.lam_s = dalloc_n<float>(ctx, (size_t)5 * ctx->n_slots);
    A.a.gadj = dalloc_n<float>(ctx, (size_t)10 * ctx->n_slots);
    A.a.padj = dalloc_n<float>(ctx, 2 * WC_MAX_PROBES);
    A.a.n_ghost_probe = q.nw + q.nd + q.n_probes;
    A.nblk = wc_adj_partial_blocks(A.a.n_ghost_probe, ctx->n_slots);
    A.a.theta_part = dalloc_n<double>(ctx, (size_t)3 * A.nblk);
    A.a.theta = dalloc_n<double>(ctx, 3);
  }
  HC(hipMemsetAsync(A.L1, 0, (size_t)5 * nf * 4, ctx->st));
  HC(hipMemsetAsync(A.a.theta, 0, 3 * 8, ctx->st));
  HC(hipMemsetAsync(A.a.theta_part, 0, (size_t)3 * A.nblk * 8, ctx->st));
  const long long steps_after = ctx->steps;
  for (int g = A.n_seg - 1; g >= 0; --g) {
    const int n = std::min(A.ckpt, A.n_steps - g * A.ckpt);
    if (!A.taped) {
      ckpt_copy(ctx, A.ckpt_dev[g], false);
      replay_taped(ctx, n);
    }
    for (int k = n - 1; k >= 0; --k) {
      const int st = g * A.ckpt + k;
      const double t = A.t[st], dt = A.dt[st];
      AdjPtrs a = A.a;
      // corrector: U^{n+1} = E_B(U^n + dt f(U*)); the enforcement transpose
      // into L0 (direct part of U^n), the rates' adjoint into Ls (U*)
      a.lam_out = A.L1;
      a.lam_base = A.L0;
      a.pre_pos = A.pB[k];
      a.pre_vel = A.vB[k];
      AdjPtrs ar = a;
      ar.lam_base = A.Ls;
      wc_enqueue_adj_eval(ctx->d, a, ar, A.tB[k], t + dt, (float)dt, false, t + 0.5 * dt, 0.0f, false, ctx->st);
      // predictor: U* = E_A(U^n + dt/2 f(U^n)); probes of step n; both
      // parts added into L0
      a.lam_out = A.Ls;
      a.lam_base = A.L0;
      a.pre_pos = A.pA[k];
      a.pre_vel = A.vA[k];
      wc_enqueue_adj_eval(ctx->d, a, a, A.tA[k], t + 0.5 * dt, (float)(0.5 * dt), true, t, (float)(dJ * dt), true,
                          ctx->st);
      HC(hipGetLastError());
      std::swap(A.L0, A.L1);
    }
  }
  wc_enqueue_adj_theta(A.a, A.nblk, ctx->st);
  HC(hipGetLastError());
  // back to the state at the end of the forward run
  ckpt_copy(ctx, A.ckpt_dev[A.n_seg], false);
  ctx->steps = steps_after;
  sync(ctx);
  HC(hipMemcpy(grad, A.a.theta, 3 * 8, hipMemcpyDeviceToHost));
  if (state_invalid(ctx, 0)) return WCSPH_E_UNSTABLE;
  API_END(ctx)
}

}  // extern "C"
