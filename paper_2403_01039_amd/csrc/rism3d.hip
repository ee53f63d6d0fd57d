// C-ABI entry points of the gfx950 3D-RISM library (see include/rism3d.h).
//
// Host orchestration only: argument checks, the workspace layout, kernel
// launches on the caller's stream and the once-per-chunk convergence poll.
// Every step of the computation runs in the kernels of setup.hpp, fft.hpp and
// iterate.hpp.

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <mutex>
#include <type_traits>
#include <vector>

#include "common.hpp"
#include "fft.hpp"
#include "iterate.hpp"
#include "forces.hpp"
#include "fused.hpp"
#include "setup.hpp"
#include "unet.hpp"

using namespace rism;

// Device scratch of rism3d_transform_noalloc: the twiddle tables of the three
// axes (2 n float2 per axis, each table 256-byte aligned), for axes of up to
// kFftMaxN points.  Every GPU the library runs on holds one copy until the
// process ends; host code reaches it only through the address that
// hipGetSymbolAddress returns for the current device.
constexpr size_t kNoAllocScratchBytes = 3 * 2 * (size_t)kFftMaxN * sizeof(float2);
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];
static_assert(kNoAllocScratchBytes == RISM3D_NOALLOC_SCRATCH_BYTES, "header size");

namespace {

thread_local std::string g_error;

rism3d_status fail(rism3d_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_error = buf;
  return s;
}

#define HIP_TRY(expr)                                                                       \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess)                                                                   \
      return fail(RISM3D_E_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));          \
  } while (0)

#define LAUNCH_CHECK()                                                                      \
  do {                                                                                      \
    hipError_t e_ = hipGetLastError();                                                      \
    if (e_ != hipSuccess)                                                                   \
      return fail(RISM3D_E_DEVICE, "kernel launch failed (%s:%d): %s", __FILE__, __LINE__, \
                  hipGetErrorString(e_));                                                   \
  } while (0)

// ---------------------------------------------------------------------------
// Optional per-family kernel timing with HIP events (thread-local).
// ---------------------------------------------------------------------------
enum Family {
  F_UPDATE32, F_UPDATE64, F_FFTX32, F_FFTY32, F_FFTZ32, F_FFTX64, F_FFTY64, F_FFTZ64,
  F_CONTRACT32, F_CONTRACT64, F_RESIDUAL32, F_RESIDUAL64, F_CONTROL, F_UPDFFT32, F_UPDFFT64,
  F_FFTRES32, F_FFTRES64, F_ZCZ32, F_ZCZ64, F_POTENTIAL, F_FTILDE, F_SETUP, F_OUTPUT, F_SFE,
  F_NET_FWD, F_NET_GRAD, F_HALFSTEP, F_SFEGRAD, F_COUNT
};
const char* const kFamilyNames[F_COUNT] = {
    "update_closure_f32", "update_closure_f64", "fft_x_f32", "fft_y_f32", "fft_z_f32",
    "fft_x_f64", "fft_y_f64", "fft_z_f64", "contract_f32", "contract_f64", "residual_gram_f32",
    "residual_gram_f64", "mdiis_control", "update_fftx_f32", "update_fftx_f64",
    "fftx_residual_f32", "fftx_residual_f64", "zfft_contract_f32", "zfft_contract_f64",
    "potential", "long_range_spectrum",
    "setup_tables", "output", "free_energy", "unet_forward", "unet_gradient", "oz_half_step",
    "sfe_gradient"};

struct Timer {
  bool on = false;
  int only = -1;   // time this family only (-1: every family)
  std::vector<hipEvent_t> pool;
  struct Pending {
    int fam;
    int tag;   // iteration index within the chunk (-1: not an iteration kernel)
    hipEvent_t a, b;
  };
  std::vector<Pending> pending;
  double ms[F_COUNT] = {};
  long count[F_COUNT] = {};
  hipEvent_t get() {
    if (pool.empty()) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      return e;
    }
    hipEvent_t e = pool.back();
    pool.pop_back();
    return e;
  }
  // Harvest completed pairs (the caller has synchronised the stream).  Only
  // iterations that executed (tag < executed) are counted: the launches that
  // follow convergence inside a chunk exit immediately.
  void harvest(int executed = 1 << 30) {
    std::vector<Pending> keep;
    for (const Pending& p : pending) {
      if (hipEventQuery(p.b) != hipSuccess) {
        keep.push_back(p);
        continue;
      }
      float t = 0.0f;
      if (p.tag < executed) {
        if (hipEventElapsedTime(&t, p.a, p.b) == hipSuccess) {
          ms[p.fam] += t;
          count[p.fam] += 1;
        } else {
          (void)hipGetLastError();
        }
      }
      pool.push_back(p.a);
      pool.push_back(p.b);
    }
    pending.swap(keep);
  }
};
thread_local Timer g_timer;
thread_local int g_iter_tag = -1;
thread_local bool g_capturing = false;     // a graph capture is in progress
thread_local bool g_capture_bad = false;   // an event node could not be added

// Records an event on s.  Under stream capture a plain hipEventRecord only
// tracks dependencies, so an explicit event-record node is appended to the
// captured graph instead; its timestamp is taken when the graph runs.
bool record_event(hipEvent_t e, hipStream_t s) {
  if (!g_capturing) return hipEventRecord(e, s) == hipSuccess;
  hipStreamCaptureStatus st;
  unsigned long long id = 0;
  hipGraph_t g = nullptr;
  const hipGraphNode_t* deps = nullptr;
  size_t nd = 0;
  hipGraphNode_t node = nullptr;
  if (hipStreamGetCaptureInfo_v2(s, &st, &id, &g, &deps, &nd) != hipSuccess ||
      st != hipStreamCaptureStatusActive ||
      hipGraphAddEventRecordNode(&node, g, deps, nd, e) != hipSuccess ||
      hipStreamUpdateCaptureDependencies(s, &node, 1, hipStreamSetCaptureDependencies) !=
          hipSuccess) {
    (void)hipGetLastError();
    g_capture_bad = true;
    return false;
  }
  return true;
}

struct TimedScope {
  hipEvent_t a = nullptr;
  int fam;
  hipStream_t s;
  TimedScope(int f, hipStream_t st) : fam(f), s(st) {
    if (g_timer.on && (g_timer.only < 0 || g_timer.only == f) && (a = g_timer.get()) &&
        !record_event(a, s)) {
      g_timer.pool.push_back(a);
      a = nullptr;
    }
  }
  ~TimedScope() {
    if (!a) return;
    hipEvent_t b = g_timer.get();
    if (!b) return;
    if (!record_event(b, s)) {
      g_timer.pool.push_back(b);
      return;   // a stays recorded and unused; it is not reused this chunk
    }
    g_timer.pending.push_back({fam, g_iter_tag, a, b});
  }
};
#define TIMED(fam, s) TimedScope timed_scope_##__LINE__(fam, s)

size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }

bool plan_axis(int n, AxisPlan* p) {
  if (n < 2 || n > kFftMaxN) return false;
  p->n = n;
  p->npass = 0;
  int m = n;
  const int radices[5] = {8, 4, 2, 3, 5};
  for (int r : radices) {
    while (m % r == 0) {
      if (p->npass >= kMaxRadixPasses) return false;
      p->radix[p->npass++] = r;
      m /= r;
    }
  }
  return m == 1;
}

double axis_kmax(int n, double dk) {
  double km = 0.0;
  for (int j = 0; j < n; ++j) {
    const double k = (2 * j < n) ? (j + 0.5) * dk : (j + 0.5 - n) * dk;
    km = fmax(km, fabs(k));
  }
  return km;
}

struct Layout {
  int nx, ny, nz, nv, npair, M, n_atoms, m_tab;
  GramW gw;   // Gram inner-product weights (1, or 1/rho for modified Anderson)
  size_t N, half;
  double dkx, dky, dkz, beta, dv;
  AxisPlan px, py, pz;
  size_t off_state, off_w, off_phi, off_F, off_tau, off_res, off_tref, off_tlo, off_rref, off_dref,
      off_dg,
      off_spec,
      off_part, off_atoms, off_lj, off_ph, off_chi32, off_chi64, off_q64, off_tw32[3], off_tw64[3],
      off_out, off_hist, total;
};

constexpr int kDefaultCheckEvery = 8;

// FNV-1a digest of what fixes the workspace offsets (grid, sites, stored
// pairs, table length, atom count, size): a workspace prepared under one
// layout and read under another (for example other MDIIS depth options) is
// refused instead of read at the wrong offsets.
unsigned layout_key(const Layout& L) {
  const unsigned long long v[8] = {(unsigned long long)L.nx, (unsigned long long)L.ny,
                                   (unsigned long long)L.nz, (unsigned long long)L.nv,
                                   (unsigned long long)L.M, (unsigned long long)L.m_tab,
                                   (unsigned long long)L.n_atoms, (unsigned long long)L.total};
  unsigned h = 2166136261u;
  for (unsigned long long x : v)
    for (int b = 0; b < 8; ++b) {
      h ^= (unsigned)((x >> (8 * b)) & 0xffu);
      h *= 16777619u;
    }
  return h;
}

rism3d_status check_prepared(const IterState& host, const Layout& L) {
  if (host.prepared != kPreparedMagic)
    return fail(RISM3D_E_WORKSPACE, "workspace not prepared: call rism3d_potential first");
  if (host.layout_key != layout_key(L))
    return fail(RISM3D_E_WORKSPACE,
                "workspace was prepared for another layout (grid, sites, MDIIS depth or "
                "accelerator, table length or atom count): call rism3d_potential with these "
                "options first");
  return RISM3D_OK;
}
// thermodynamic results left in the workspace by launch_sfe: per-site free
// energies, their total, per-site rho_g \int c_g
constexpr int kOutDoubles = 2 * kMaxSites + 1;
constexpr int kDefaultAnchorEvery = 32;

rism3d_status make_layout(const rism3d_problem* pr, const rism3d_opts* op, Layout* L) {
  if (!pr || !op) return fail(RISM3D_E_ARG, "null problem or options");
  if (pr->n_atoms < 0) return fail(RISM3D_E_ARG, "n_atoms < 0");
  if (pr->n_atoms > 0 && (!pr->xyz || !pr->q || !pr->sigma || !pr->eps))
    return fail(RISM3D_E_ARG, "null solute atom array");
  if (pr->n_sites < 1 || pr->n_sites > kMaxSites)
    return fail(RISM3D_E_ARG, "n_sites must be in 1..%d", kMaxSites);
  if (!pr->site_q || !pr->site_sigma || !pr->site_eps || !pr->site_rho)
    return fail(RISM3D_E_ARG, "null solvent site array");
  for (int g = 0; g < pr->n_sites; ++g) {
    if (!(pr->site_rho[g] > 0.0) || !(pr->site_sigma[g] >= 0.0) || !(pr->site_eps[g] >= 0.0))
      return fail(RISM3D_E_ARG, "invalid parameters for solvent site %d", g);
  }
  if (pr->n_k < 2 || !(pr->dk > 0.0) || !pr->chi)
    return fail(RISM3D_E_ARG, "invalid susceptibility table (n_k, dk, chi)");
  if (!(pr->temperature > 0.0)) return fail(RISM3D_E_ARG, "temperature must be > 0");
  if (!(pr->spacing > 0.0)) return fail(RISM3D_E_ARG, "spacing must be > 0");
  if (!(pr->compressibility >= 0.0) || !std::isfinite(pr->compressibility) ||
      !std::isfinite(pr->pressure))
    return fail(RISM3D_E_ARG, "compressibility must be finite and >= 0, pressure finite");
  if (!plan_axis(pr->nx, &L->px) || !plan_axis(pr->ny, &L->py) || !plan_axis(pr->nz, &L->pz) ||
      (pr->nx | pr->ny | pr->nz) & 1)
    return fail(RISM3D_E_ARG,
                "grid %dx%dx%d unsupported: each axis must be even, 2..%d, with prime factors "
                "2, 3, 5 (an odd axis has a self-mirrored half-integer frequency where the "
                "analytic long-range spectrum is not Hermitian)",
                pr->nx, pr->ny, pr->nz, kFftMaxN);
  if (op->closure != RISM3D_KH && op->closure != RISM3D_HNC && op->closure != RISM3D_PSE)
    return fail(RISM3D_E_ARG, "unknown closure %d", (int)op->closure);
  if (op->closure == RISM3D_PSE && (op->pse_order < 1 || op->pse_order > 16))
    return fail(RISM3D_E_ARG, "pse_order must be in 1..16");
  if (!(op->tol > 0.0)) return fail(RISM3D_E_ARG, "tol must be > 0");
  if (op->max_iter < 1) return fail(RISM3D_E_ARG, "max_iter must be >= 1");
  if (op->mdiis_depth < 1 || op->mdiis_depth > kMaxDepth)
    return fail(RISM3D_E_ARG, "mdiis_depth must be in 1..%d", kMaxDepth);
  if (!(op->mdiis_eta > 0.0) || op->mdiis_eta > 2.0)
    return fail(RISM3D_E_ARG, "mdiis_eta must be in (0, 2]");
  if (op->check_every < 0 || op->anchor_every < 0)
    return fail(RISM3D_E_ARG, "check_every and anchor_every must be >= 0");
  if (op->accelerator != RISM3D_MDIIS && op->accelerator != RISM3D_ANDERSON)
    return fail(RISM3D_E_ARG, "unknown accelerator %d", (int)op->accelerator);
  if (op->accelerator == RISM3D_ANDERSON &&
      !(std::isfinite(op->anderson_s1) && std::isfinite(op->anderson_s2)))
    return fail(RISM3D_E_ARG, "anderson_s1 and anderson_s2 must be finite");

  L->nx = pr->nx;
  L->ny = pr->ny;
  L->nz = pr->nz;
  L->nv = pr->n_sites;
  L->npair = (pr->n_sites + 1) / 2;
  // modified Anderson keeps the newest input/output pair and two histories
  L->M = op->accelerator == RISM3D_ANDERSON ? 3 : op->mdiis_depth;
  for (int g = 0; g < kMaxSites; ++g)
    L->gw.w[g] = (op->accelerator == RISM3D_ANDERSON && g < pr->n_sites)
                     ? (float)(1.0 / pr->site_rho[g]) : 1.0f;
  L->n_atoms = pr->n_atoms;
  L->N = (size_t)pr->nx * pr->ny * pr->nz;
  L->half = (L->N + 1) / 2;
  const double two_pi = 6.283185307179586476925286766559;
  L->dkx = two_pi / (pr->nx * pr->spacing);
  L->dky = two_pi / (pr->ny * pr->spacing);
  L->dkz = two_pi / (pr->nz * pr->spacing);
  L->beta = 1.0 / (kBoltzmann * pr->temperature);
  L->dv = pr->spacing * pr->spacing * pr->spacing;
  const double kx = axis_kmax(pr->nx, L->dkx), ky = axis_kmax(pr->ny, L->dky),
               kz = axis_kmax(pr->nz, L->dkz);
  const double kmax = sqrt(kx * kx + ky * ky + kz * kz);
  const double mmax = kmax / pr->dk;
  if (mmax > (double)(pr->n_k - 1))
    return fail(RISM3D_E_ARG, "susceptibility table ends at k=%g but the grid reaches |k|=%g",
                (pr->n_k - 1) * pr->dk, kmax);
  L->m_tab = (int)fmin((double)pr->n_k, floor(mmax) + 3.0);
  if (L->m_tab < 2) L->m_tab = 2;

  const size_t nv = L->nv, N = L->N, M = L->M;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align_up(off + bytes);
    return o;
  };
  L->off_state = take(sizeof(IterState));
  L->off_w = take(nv * N * sizeof(float));
  L->off_phi = take(N * sizeof(float));
  L->off_F = take(L->half * sizeof(double2));
  L->off_tau = take(M * nv * N * sizeof(float));
  L->off_res = take(M * nv * N * sizeof(float));
  L->off_tref = take(nv * N * sizeof(float));
  L->off_tlo = take(nv * N * sizeof(float));
  L->off_rref = take(nv * N * sizeof(float));
  L->off_dref = take(nv * N * sizeof(float));
  L->off_dg = take(nv * N * sizeof(float));
  L->off_spec = take((size_t)L->npair * N * sizeof(double2));   // float2 in the bulk iterations
  const size_t part_q = (size_t)((M + 1) > 2 * nv ? (M + 1) : 2 * nv);
  size_t part_blocks = kRedBlocks;
  if (fixed_fft_size(pr->nx)) {   // one partial row per workgroup of the fused residual
    // (the narrowest variant: the FP64 tile, or 8 rows for a tuned FP32 one)
    size_t lines = (size_t)(2048 / pr->nx > 1 ? 2048 / pr->nx : 1);
    if (lines > 8) lines = 8;
    const size_t b = ((size_t)L->npair * pr->nz * pr->ny + lines - 1) / lines;
    if (b > part_blocks) part_blocks = b;
  }
  L->off_part = take(part_blocks * part_q * sizeof(double));
  L->off_chi32 = take((size_t)L->m_tab * chi_row<float>((int)nv) * sizeof(float));
  L->off_chi64 = take((size_t)L->m_tab * chi_row<double>((int)nv) * sizeof(double));
  L->off_q64 = take((size_t)L->m_tab * nv * sizeof(double));
  const int dims[3] = {pr->nx, pr->ny, pr->nz};
  for (int a = 0; a < 3; ++a) {
    L->off_tw32[a] = take(2 * (size_t)dims[a] * sizeof(float2));
    L->off_tw64[a] = take(2 * (size_t)dims[a] * sizeof(double2));
  }
  L->off_out = take(kOutDoubles * sizeof(double));
  L->off_hist = take(kHistLen * sizeof(double2));
  // Solute-size dependent regions last: every offset above depends only on the
  // grid, the sites, the MDIIS depth and the table length, so solves of
  // different solutes on one grid share the offsets the iteration reads.
  const size_t na = pr->n_atoms > 0 ? (size_t)pr->n_atoms : 1;
  L->off_atoms = take(na * sizeof(double4));
  L->off_lj = take(na * nv * sizeof(double2));
  L->off_ph = take(na * (size_t)(pr->nx + pr->ny + pr->nz) * sizeof(double2));
  L->total = off;
  return RISM3D_OK;
}

rism3d_status check_ws(const Layout& L, const void* ws, size_t bytes) {
  if (!ws) return fail(RISM3D_E_WORKSPACE, "null workspace");
  if (((uintptr_t)ws) & 255) return fail(RISM3D_E_WORKSPACE, "workspace must be 256-byte aligned");
  if (bytes < L.total)
    return fail(RISM3D_E_WORKSPACE, "workspace holds %zu bytes, %zu needed", bytes, L.total);
  return RISM3D_OK;
}

template <typename T>
T* at(void* ws, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(ws) + off);
}
template <typename T>
const T* at(const void* ws, size_t off) {
  return reinterpret_cast<const T*>(static_cast<const char*>(ws) + off);
}

SiteConsts site_consts(const rism3d_problem* pr, double beta) {
  SiteConsts sc;
  memset(&sc, 0, sizeof(sc));
  sc.nv = pr->n_sites;
  for (int g = 0; g < pr->n_sites; ++g) {
    sc.coul[g] = (float)(beta * kCoulomb * pr->site_q[g]);
    sc.coul64[g] = beta * kCoulomb * pr->site_q[g];
    sc.q64[g] = pr->site_q[g];
    sc.rho[g] = pr->site_rho[g];
  }
  return sc;
}

unsigned blocks_for(size_t n, int threads) { return (unsigned)((n + threads - 1) / threads); }

template <int NV>
void launch_potential_nv(const Layout& L, void* ws, double dr, const SiteConsts& sc,
                         hipStream_t s) {
  {
    TIMED(F_POTENTIAL, s);
    hipLaunchKernelGGL(k_potential<NV>, dim3(blocks_for(L.N, kPotThreads)), dim3(kPotThreads), 0, s,
                       at<double4>(ws, L.off_atoms), at<double2>(ws, L.off_lj), L.n_atoms, L.nx, L.ny,
                       L.nz, dr, sc, at<float>(ws, L.off_w), at<float>(ws, L.off_phi));
  }
}

void launch_potential(const Layout& L, void* ws, double dr, const SiteConsts& sc, hipStream_t s) {
  switch (L.nv) {
    case 1: launch_potential_nv<1>(L, ws, dr, sc, s); break;
    case 2: launch_potential_nv<2>(L, ws, dr, sc, s); break;
    case 3: launch_potential_nv<3>(L, ws, dr, sc, s); break;
    case 4: launch_potential_nv<4>(L, ws, dr, sc, s); break;
    case 5: launch_potential_nv<5>(L, ws, dr, sc, s); break;
    case 6: launch_potential_nv<6>(L, ws, dr, sc, s); break;
    case 7: launch_potential_nv<7>(L, ws, dr, sc, s); break;
    default: launch_potential_nv<8>(L, ws, dr, sc, s); break;
  }
}

template <int NV>
void launch_contract_nv(const Layout& L, void* ws, bool anchor, double inv_dkt, const int* done,
                        hipStream_t s) {
  const dim3 grid(blocks_for(L.half, kElemThreads)), block(kElemThreads);
  if (anchor)
    {
      TIMED(F_CONTRACT64, s);
      hipLaunchKernelGGL((k_contract<NV, double2, true>), grid, block, 0, s,
                         at<double2>(ws, L.off_spec), L.nx, L.ny, L.nz, L.dkx, L.dky,
                         L.dkz, at<double2>(ws, L.off_F), at<double>(ws, L.off_chi64),
                         at<double>(ws, L.off_q64), inv_dkt, L.m_tab, done);
    }
  else
    {
      TIMED(F_CONTRACT32, s);
      hipLaunchKernelGGL((k_contract<NV, float2, false>), grid, block, 0, s,
                         at<float2>(ws, L.off_spec), L.nx, L.ny, L.nz, L.dkx, L.dky,
                         L.dkz, (const float2*)nullptr, at<float>(ws, L.off_chi32),
                         (const float*)nullptr, inv_dkt, L.m_tab, done);
    }
}

void launch_contract(const Layout& L, void* ws, bool anchor, double inv_dkt, const int* done,
                     hipStream_t s) {
  switch (L.nv) {
    case 1: launch_contract_nv<1>(L, ws, anchor, inv_dkt, done, s); break;
    case 2: launch_contract_nv<2>(L, ws, anchor, inv_dkt, done, s); break;
    case 3: launch_contract_nv<3>(L, ws, anchor, inv_dkt, done, s); break;
    case 4: launch_contract_nv<4>(L, ws, anchor, inv_dkt, done, s); break;
    case 5: launch_contract_nv<5>(L, ws, anchor, inv_dkt, done, s); break;
    case 6: launch_contract_nv<6>(L, ws, anchor, inv_dkt, done, s); break;
    case 7: launch_contract_nv<7>(L, ws, anchor, inv_dkt, done, s); break;
    default: launch_contract_nv<8>(L, ws, anchor, inv_dkt, done, s); break;
  }
}

// A batched launch covers nb members whose workspaces lie stride bytes apart
// (blockIdx.y selects the member); a single solve is {1, 0}.
struct Batch {
  int nb = 1;
  size_t stride = 0;
};

// Tile choices of the autotuner, per (nx, ny, nz, sites): y-pass lines per
// workgroup and z-kernel columns per workgroup of the FP32 iterations (0 =
// the compiled default).  They change which workgroup transforms a line, not
// the operations on it (results agree to round-off).
struct Tune {
  int y_lines = 0;
  int z_cols = 0;
  int x_lines = 0;   // rows per workgroup of the fused x kernels
};
std::mutex g_tune_mu;
std::vector<std::pair<std::array<int, 4>, Tune>> g_tunes;

Tune tune_for(const Layout& L) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  for (const auto& e : g_tunes)
    if (e.first == std::array<int, 4>{L.nx, L.ny, L.nz, L.nv}) return e.second;
  return Tune{};
}

void set_tune(const Layout& L, Tune t) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  for (auto& e : g_tunes)
    if (e.first == std::array<int, 4>{L.nx, L.ny, L.nz, L.nv}) {
      e.second = t;
      return;
    }
  g_tunes.push_back({std::array<int, 4>{L.nx, L.ny, L.nz, L.nv}, t});
}

template <typename C, int N, int AXIS, int LINES = fixed_lines<C, N, AXIS>()>
void launch_fixed_n(const Layout& L, C* spec, const C* tw, int forward, const int* done,
                    hipStream_t s, Batch bt = {}) {
  unsigned grid;
  if (AXIS == 0) {
    const size_t rows = (size_t)L.npair * L.nz * L.ny;
    grid = (unsigned)((rows + LINES - 1) / LINES);
  } else {
    const int tiles_x = (L.nx + LINES - 1) / LINES;
    const int outer = AXIS == 1 ? L.npair * L.nz : L.npair * L.ny;
    grid = (unsigned)outer * tiles_x;
  }
  hipLaunchKernelGGL((k_fft_fixed<C, N, AXIS, LINES>), dim3(grid, bt.nb), dim3(kFftThreads), 0, s,
                     spec, L.nx, L.ny, L.nz, L.npair, tw, forward, done, bt.stride);
}

// y pass of the FP32 iterations with a tuned width (lines = 0: default).
template <int N>
void launch_y32_n(const Layout& L, float2* spec, const float2* tw, int forward, const int* done,
                  hipStream_t s, Batch bt, int lines) {
  switch (lines) {
    case 8: launch_fixed_n<float2, N, 1, 8>(L, spec, tw, forward, done, s, bt); break;
    case 16: launch_fixed_n<float2, N, 1, 16>(L, spec, tw, forward, done, s, bt); break;
    case 32:
      if constexpr (N <= 256) {
        launch_fixed_n<float2, N, 1, 32>(L, spec, tw, forward, done, s, bt);
        break;
      }
      [[fallthrough]];
    case 64:
      if constexpr (N <= 128) {
        launch_fixed_n<float2, N, 1, 64>(L, spec, tw, forward, done, s, bt);
        break;
      }
      [[fallthrough]];
    default: launch_fixed_n<float2, N, 1>(L, spec, tw, forward, done, s, bt); break;
  }
}

bool launch_y32(const Layout& L, float2* spec, const float2* tw, int forward, const int* done,
                hipStream_t s, Batch bt, int lines) {
  TIMED(F_FFTY32, s);
  switch (L.ny) {
    case 32: launch_y32_n<32>(L, spec, tw, forward, done, s, bt, lines); return true;
    case 64: launch_y32_n<64>(L, spec, tw, forward, done, s, bt, lines); return true;
    case 96: launch_y32_n<96>(L, spec, tw, forward, done, s, bt, lines); return true;
    case 128: launch_y32_n<128>(L, spec, tw, forward, done, s, bt, lines); return true;
    case 192: launch_y32_n<192>(L, spec, tw, forward, done, s, bt, lines); return true;
    case 256: launch_y32_n<256>(L, spec, tw, forward, done, s, bt, lines); return true;
    case 512: launch_y32_n<512>(L, spec, tw, forward, done, s, bt, lines); return true;
    default: return false;
  }
}

template <typename C, int AXIS>
bool launch_fixed_axis(int n, const Layout& L, C* spec, const C* tw, int forward, const int* done,
                       hipStream_t s, Batch bt) {
  switch (n) {
    case 32: launch_fixed_n<C, 32, AXIS>(L, spec, tw, forward, done, s, bt); return true;
    case 64: launch_fixed_n<C, 64, AXIS>(L, spec, tw, forward, done, s, bt); return true;
    case 96: launch_fixed_n<C, 96, AXIS>(L, spec, tw, forward, done, s, bt); return true;
    case 128: launch_fixed_n<C, 128, AXIS>(L, spec, tw, forward, done, s, bt); return true;
    case 192: launch_fixed_n<C, 192, AXIS>(L, spec, tw, forward, done, s, bt); return true;
    case 256: launch_fixed_n<C, 256, AXIS>(L, spec, tw, forward, done, s, bt); return true;
    case 512: launch_fixed_n<C, 512, AXIS>(L, spec, tw, forward, done, s, bt); return true;
    default: return false;
  }
}

// One axis pass of the shifted transform over all packed pairs.
template <typename C>
void launch_axis(const Layout& L, C* spec, const C* const tw[3], int axis, int forward,
                 const int* done, hipStream_t s, Batch bt = {}) {
  const bool f64 = std::is_same<C, double2>::value;
  const AxisPlan& p = axis == 0 ? L.px : (axis == 1 ? L.py : L.pz);
  TIMED((f64 ? F_FFTX64 : F_FFTX32) + axis, s);
  bool ok = false;
  if (fixed_fft_size(p.n)) {
    if (axis == 0) ok = launch_fixed_axis<C, 0>(p.n, L, spec, tw[axis], forward, done, s, bt);
    else if (axis == 1) ok = launch_fixed_axis<C, 1>(p.n, L, spec, tw[axis], forward, done, s, bt);
    else ok = launch_fixed_axis<C, 2>(p.n, L, spec, tw[axis], forward, done, s, bt);
  }
  if (ok) return;   // batches only reach here with fixed-size lengths (batch_plan)
  const int lines = fft_lines_per_block<C>(axis, p.n, L.nx);
  unsigned grid;
  if (axis == 0) {
    const size_t rows = (size_t)L.npair * L.nz * L.ny;
    grid = (unsigned)((rows + lines - 1) / lines);
  } else {
    const int tiles_x = (L.nx + lines - 1) / lines;
    const int outer = axis == 1 ? L.npair * L.nz : L.npair * L.ny;
    grid = (unsigned)outer * tiles_x;
  }
  hipLaunchKernelGGL(k_fft_axis<C>, dim3(grid), dim3(kFftThreads), 0, s, spec, L.nx, L.ny, L.nz,
                     L.npair, axis, p, tw[axis], forward, lines, done);
}

// Forward (forward != 0) or inverse 3D transform of all packed pairs, one
// kernel per axis; C = float2 (bulk) or double2 (anchor).  Common lengths use
// the fixed-size kernels, others the generic runtime-plan kernel.
template <typename C>
void launch_fft3_on(const Layout& L, C* spec, const C* const tw[3], int forward, const int* done,
                    hipStream_t s, bool skip_x = false) {
  const int axes_fwd[3] = {0, 1, 2};
  const int axes_inv[3] = {2, 1, 0};
  for (int k = 0; k < 3; ++k) {
    const int axis = forward ? axes_fwd[k] : axes_inv[k];
    if (skip_x && axis == 0) continue;
    launch_axis(L, spec, tw, axis, forward, done, s);
  }
}

template <typename C>
void launch_fft3(const Layout& L, void* ws, int forward, const int* done, hipStream_t s,
                 bool skip_x = false);

template <>
void launch_fft3<float2>(const Layout& L, void* ws, int forward, const int* done, hipStream_t s,
                         bool skip_x) {
  const float2* tw[3] = {at<float2>(ws, L.off_tw32[0]), at<float2>(ws, L.off_tw32[1]),
                         at<float2>(ws, L.off_tw32[2])};
  launch_fft3_on(L, at<float2>(ws, L.off_spec), tw, forward, done, s, skip_x);
}

template <>
void launch_fft3<double2>(const Layout& L, void* ws, int forward, const int* done, hipStream_t s,
                          bool skip_x) {
  const double2* tw[3] = {at<double2>(ws, L.off_tw64[0]), at<double2>(ws, L.off_tw64[1]),
                          at<double2>(ws, L.off_tw64[2])};
  launch_fft3_on(L, at<double2>(ws, L.off_spec), tw, forward, done, s, skip_x);
}

// Fused z transform + contraction + inverse z transform.
bool zcz_supported(const Layout& L) {
  return (L.ny % 2) == 0 && (L.nz == 64 || L.nz == 96 || L.nz == 128 || L.nz == 256);
}

template <typename C, int NZ, int NV, int B = zcz_cols<C, NZ, NV>()>
void launch_zcz_b(const Layout& L, void* ws, double inv_dkt, const int* done, hipStream_t s,
                  Batch bt) {
  constexpr bool F64 = std::is_same<C, double2>::value;
  const int tiles_x = (L.nx + B - 1) / B;
  const dim3 grid((unsigned)(L.ny / 2) * tiles_x, bt.nb), block(kFftThreads);
  using S = typename ScalarOf<C>::type;
  TIMED(F64 ? F_ZCZ64 : F_ZCZ32, s);
  hipLaunchKernelGGL((k_zcz<C, NZ, NV, F64, B>), grid, block, 0, s, at<C>(ws, L.off_spec), L.nx,
                     L.ny, at<C>(ws, F64 ? L.off_tw64[2] : L.off_tw32[2]), L.dkx,
                     L.dky, L.dkz, F64 ? at<C>(ws, L.off_F) : (const C*)nullptr,
                     at<S>(ws, F64 ? L.off_chi64 : L.off_chi32),
                     F64 ? at<S>(ws, L.off_q64) : (const S*)nullptr, inv_dkt, L.m_tab, done,
                     bt.stride);
}

// FP32 z kernel with a tuned width (cols = 0: default); widths whose tile
// would exceed 120 KB of LDS are not compiled and fall back to the default.
template <typename C, int NZ, int NV>
void launch_zcz_n(const Layout& L, void* ws, double inv_dkt, const int* done, hipStream_t s,
                  Batch bt, int cols = 0) {
  if constexpr (std::is_same<C, float2>::value) {
    constexpr int per_col = 2 * ((NV + 1) / 2) * Lds<NZ>::PITCH * (int)sizeof(C);
    if (cols == 4) { launch_zcz_b<C, NZ, NV, 4>(L, ws, inv_dkt, done, s, bt); return; }
    if constexpr (per_col * 8 <= 122880)
      if (cols == 8) { launch_zcz_b<C, NZ, NV, 8>(L, ws, inv_dkt, done, s, bt); return; }
    if constexpr (per_col * 16 <= 122880)
      if (cols == 16) { launch_zcz_b<C, NZ, NV, 16>(L, ws, inv_dkt, done, s, bt); return; }
  }
  launch_zcz_b<C, NZ, NV>(L, ws, inv_dkt, done, s, bt);
}

template <typename C, int NZ>
void launch_zcz_nz(const Layout& L, void* ws, double inv_dkt, const int* done, hipStream_t s,
                   Batch bt, int cols) {
  switch (L.nv) {
    case 1: launch_zcz_n<C, NZ, 1>(L, ws, inv_dkt, done, s, bt, cols); break;
    case 2: launch_zcz_n<C, NZ, 2>(L, ws, inv_dkt, done, s, bt, cols); break;
    case 3: launch_zcz_n<C, NZ, 3>(L, ws, inv_dkt, done, s, bt, cols); break;
    case 4: launch_zcz_n<C, NZ, 4>(L, ws, inv_dkt, done, s, bt, cols); break;
    case 5: launch_zcz_n<C, NZ, 5>(L, ws, inv_dkt, done, s, bt, cols); break;
    case 6: launch_zcz_n<C, NZ, 6>(L, ws, inv_dkt, done, s, bt, cols); break;
    case 7: launch_zcz_n<C, NZ, 7>(L, ws, inv_dkt, done, s, bt, cols); break;
    default: launch_zcz_n<C, NZ, 8>(L, ws, inv_dkt, done, s, bt, cols); break;
  }
}

template <typename C>
void launch_zcz(const Layout& L, void* ws, double inv_dkt, const int* done, hipStream_t s,
                Batch bt, int cols = 0) {
  switch (L.nz) {
    case 64: launch_zcz_nz<C, 64>(L, ws, inv_dkt, done, s, bt, cols); break;
    case 96: launch_zcz_nz<C, 96>(L, ws, inv_dkt, done, s, bt, cols); break;
    case 128: launch_zcz_nz<C, 128>(L, ws, inv_dkt, done, s, bt, cols); break;
    default: launch_zcz_nz<C, 256>(L, ws, inv_dkt, done, s, bt, cols); break;
  }
}

// Fused first and last kernels of an iteration (x-axis transform fused with the
// update+closure and with the residual+Gram+control).
template <bool ANCHOR, int N, int LINES = fixed_lines<PrecC<ANCHOR>, N, 0>()>
void launch_fused_l(const Layout& L, void* ws, const rism3d_opts* op, bool first_half,
                    hipStream_t s, Batch bt, bool control) {
  using C = PrecC<ANCHOR>;
  IterState* st = at<IterState>(ws, L.off_state);
  const int kind = (int)op->closure;
  const int order = op->closure == RISM3D_PSE ? op->pse_order : 1;
  const size_t rows = (size_t)L.npair * L.nz * L.ny;
  const dim3 grid((unsigned)((rows + LINES - 1) / LINES), bt.nb), block(kFftThreads);
  const C* tw = at<C>(ws, ANCHOR ? L.off_tw64[0] : L.off_tw32[0]);
  if (first_half) {
    TIMED(ANCHOR ? F_UPDFFT64 : F_UPDFFT32, s);
    auto update = &k_update_fftx<ANCHOR, N, LINES, kMaxDepth>;
    if constexpr (!ANCHOR) {
      if (L.M <= 3) update = &k_update_fftx<false, N, LINES, 3>;
      else if (L.M <= 5) update = &k_update_fftx<false, N, LINES, 5>;
    }
    hipLaunchKernelGGL(update, grid, block, 0, s, st,
                       at<float>(ws, L.off_tau), at<float>(ws, L.off_res), at<float>(ws, L.off_w),
                       at<float>(ws, L.off_tref), at<float>(ws, L.off_tlo),
                       at<float>(ws, L.off_dref), at<float>(ws, L.off_dg),
                       at<void>(ws, L.off_spec), L.ny, L.nz, L.nv, L.npair, L.M, kind, order, tw,
                       bt.stride);
  } else {
    {
      TIMED(ANCHOR ? F_FFTRES64 : F_FFTRES32, s);
      // the FP32 residual holds one Gram accumulator per possible slot: a
      // tight bound for the usual depths keeps registers (and occupancy) free
      auto residual = &k_fftx_residual<ANCHOR, N, LINES, kMaxDepth>;
      if constexpr (!ANCHOR) {
        if (L.M <= 3) residual = &k_fftx_residual<false, N, LINES, 3>;
        else if (L.M <= 5) residual = &k_fftx_residual<false, N, LINES, 5>;
      }
      hipLaunchKernelGGL(residual, grid, block, 0, s, st,
                         at<void>(ws, L.off_spec), at<float>(ws, L.off_w),
                         at<float>(ws, L.off_tau), at<float>(ws, L.off_res),
                         at<float>(ws, L.off_tref), at<float>(ws, L.off_tlo),
                         at<float>(ws, L.off_rref), at<float>(ws, L.off_dref),
                         at<float>(ws, L.off_dg), L.ny, L.nz, L.nv, L.npair, L.M, kind, order, tw,
                         at<double>(ws, L.off_part), L.gw, bt.stride);
    }
    if (!control) return;
    TIMED(F_CONTROL, s);
    const double inv_count = 1.0 / ((double)L.N * (double)L.nv);
    hipLaunchKernelGGL(L.M <= 5 ? &k_control<5> : &k_control<kMaxDepth>, dim3(1, bt.nb),
                       dim3(kCtlThreads), 0, s, st,
                       at<double>(ws, L.off_part), (int)grid.x, L.M, inv_count, op->tol,
                       op->max_iter, (float)op->mdiis_eta, op->eta_dynamic,
                       (int)op->accelerator, op->anderson_s1, op->anderson_s2, ANCHOR ? 1 : 0,
                       at<double2>(ws, L.off_hist), bt.stride);
  }
}

// FP32 fused kernels with a tuned row count (lines = 0: default); counts
// whose LDS tile would exceed 64 KB are not compiled and run the default.
template <bool ANCHOR, int N>
void launch_fused_n(const Layout& L, void* ws, const rism3d_opts* op, bool first_half,
                    hipStream_t s, Batch bt, int lines, bool control) {
  if constexpr (!ANCHOR) {
    constexpr int row = Lds<N>::PITCH * (int)sizeof(float2);
    if (lines == 8) {
      launch_fused_l<false, N, 8>(L, ws, op, first_half, s, bt, control);
      return;
    }
    if constexpr (16 * row <= 65536)
      if (lines == 16) {
        launch_fused_l<false, N, 16>(L, ws, op, first_half, s, bt, control);
        return;
      }
    if constexpr (32 * row <= 65536)
      if (lines == 32) {
        launch_fused_l<false, N, 32>(L, ws, op, first_half, s, bt, control);
        return;
      }
  }
  launch_fused_l<ANCHOR, N>(L, ws, op, first_half, s, bt, control);
}

// control = false leaves out the MDIIS control launch after the residual
// kernel (the autotuner times the two fused kernels alone).
template <bool ANCHOR>
void launch_fused(const Layout& L, void* ws, const rism3d_opts* op, bool first_half,
                  hipStream_t s, Batch bt, int lines = 0, bool control = true) {
  switch (L.nx) {
    case 32: launch_fused_n<ANCHOR, 32>(L, ws, op, first_half, s, bt, lines, control); break;
    case 64: launch_fused_n<ANCHOR, 64>(L, ws, op, first_half, s, bt, lines, control); break;
    case 96: launch_fused_n<ANCHOR, 96>(L, ws, op, first_half, s, bt, lines, control); break;
    case 128: launch_fused_n<ANCHOR, 128>(L, ws, op, first_half, s, bt, lines, control); break;
    case 192: launch_fused_n<ANCHOR, 192>(L, ws, op, first_half, s, bt, lines, control); break;
    case 256: launch_fused_n<ANCHOR, 256>(L, ws, op, first_half, s, bt, lines, control); break;
    default: launch_fused_n<ANCHOR, 512>(L, ws, op, first_half, s, bt, lines, control); break;
  }
}

// One evaluation of the 3D-RISM map plus the MDIIS bookkeeping: update +
// closure, forward FFT, contraction, inverse FFT, residual + Gram row, control.
// anchor: FP64 evaluation that re-bases the FP32 increments.
void launch_iteration(const Layout& L, void* ws, const rism3d_opts* op, double inv_dkt,
                      bool anchor, hipStream_t s, Batch bt = {}) {
  IterState* st = at<IterState>(ws, L.off_state);
  const int* done = &st->done;
  const int kind = (int)op->closure;
  const int order = op->closure == RISM3D_PSE ? op->pse_order : 1;
  if (fixed_fft_size(L.nx)) {
    const int xl = anchor ? 0 : tune_for(L).x_lines;
    if (anchor) launch_fused<true>(L, ws, op, true, s, bt);
    else launch_fused<false>(L, ws, op, true, s, bt, xl);
    if (zcz_supported(L)) {
      // y pass, then z + contraction + z fused, then inverse y pass
      const float2* tw32[3] = {at<float2>(ws, L.off_tw32[0]), at<float2>(ws, L.off_tw32[1]),
                               at<float2>(ws, L.off_tw32[2])};
      const double2* tw64[3] = {at<double2>(ws, L.off_tw64[0]), at<double2>(ws, L.off_tw64[1]),
                                at<double2>(ws, L.off_tw64[2])};
      if (anchor) {
        launch_axis(L, at<double2>(ws, L.off_spec), tw64, 1, 1, done, s, bt);
        launch_zcz<double2>(L, ws, inv_dkt, done, s, bt);
        launch_axis(L, at<double2>(ws, L.off_spec), tw64, 1, 0, done, s, bt);
      } else {
        const Tune tn = tune_for(L);
        if (!launch_y32(L, at<float2>(ws, L.off_spec), tw32[1], 1, done, s, bt, tn.y_lines))
          launch_axis(L, at<float2>(ws, L.off_spec), tw32, 1, 1, done, s, bt);
        launch_zcz<float2>(L, ws, inv_dkt, done, s, bt, tn.z_cols);
        if (!launch_y32(L, at<float2>(ws, L.off_spec), tw32[1], 0, done, s, bt, tn.y_lines))
          launch_axis(L, at<float2>(ws, L.off_spec), tw32, 1, 0, done, s, bt);
      }
    } else {
      if (anchor) launch_fft3<double2>(L, ws, 1, done, s, true);
      else launch_fft3<float2>(L, ws, 1, done, s, true);
      launch_contract(L, ws, anchor, inv_dkt, done, s);
      if (anchor) launch_fft3<double2>(L, ws, 0, done, s, true);
      else launch_fft3<float2>(L, ws, 0, done, s, true);
    }
    if (anchor) launch_fused<true>(L, ws, op, false, s, bt);
    else launch_fused<false>(L, ws, op, false, s, bt, xl);
    return;
  }
  const bool v4 = (L.N % 4) == 0;
  const size_t quads = (size_t)L.npair * (v4 ? L.N / 4 : L.N);
  const dim3 eg(blocks_for(quads, kElemThreads)), eb(kElemThreads);
#define RISM_UPDATE_ARGS                                                                    \
  st, at<float>(ws, L.off_tau), at<float>(ws, L.off_res), at<float>(ws, L.off_w),     \
      at<float>(ws, L.off_tref), at<float>(ws, L.off_tlo), at<float>(ws, L.off_dref),         \
      at<float>(ws, L.off_dg), at<void>(ws, L.off_spec), L.N, L.nv, L.npair, L.M, kind, order
  {
    TIMED(anchor ? F_UPDATE64 : F_UPDATE32, s);
    if (anchor && v4) hipLaunchKernelGGL((k_update_closure<true, 4>), eg, eb, 0, s, RISM_UPDATE_ARGS);
    else if (anchor) hipLaunchKernelGGL((k_update_closure<true, 1>), eg, eb, 0, s, RISM_UPDATE_ARGS);
    else if (v4) hipLaunchKernelGGL((k_update_closure<false, 4>), eg, eb, 0, s, RISM_UPDATE_ARGS);
    else hipLaunchKernelGGL((k_update_closure<false, 1>), eg, eb, 0, s, RISM_UPDATE_ARGS);
  }
#undef RISM_UPDATE_ARGS
  if (anchor) launch_fft3<double2>(L, ws, 1, done, s);
  else launch_fft3<float2>(L, ws, 1, done, s);
  launch_contract(L, ws, anchor, inv_dkt, done, s);
  if (anchor) launch_fft3<double2>(L, ws, 0, done, s);
  else launch_fft3<float2>(L, ws, 0, done, s);
  unsigned nblk = blocks_for(quads, kRedThreads);
  if (nblk > (unsigned)kRedBlocks) nblk = kRedBlocks;
#define RISM_RESID_ARGS                                                                       \
  st, at<void>(ws, L.off_spec), at<float>(ws, L.off_w), at<float>(ws, L.off_tau),             \
      at<float>(ws, L.off_res), at<float>(ws, L.off_tref), at<float>(ws, L.off_tlo),          \
      at<float>(ws, L.off_rref), at<float>(ws, L.off_dref), at<float>(ws, L.off_dg), L.N, L.nv,  \
      L.npair, L.M, kind, order,                                                                \
      at<double>(ws, L.off_part), L.gw
  {
    TIMED(anchor ? F_RESIDUAL64 : F_RESIDUAL32, s);
    const dim3 rg(nblk), rb(kRedThreads);
    if (anchor && v4) hipLaunchKernelGGL((k_residual<true, 4>), rg, rb, 0, s, RISM_RESID_ARGS);
    else if (anchor) hipLaunchKernelGGL((k_residual<true, 1>), rg, rb, 0, s, RISM_RESID_ARGS);
    else if (v4) hipLaunchKernelGGL((k_residual<false, 4>), rg, rb, 0, s, RISM_RESID_ARGS);
    else hipLaunchKernelGGL((k_residual<false, 1>), rg, rb, 0, s, RISM_RESID_ARGS);
  }
#undef RISM_RESID_ARGS
  const double inv_count = 1.0 / ((double)L.N * (double)L.nv);
  {
    TIMED(F_CONTROL, s);
    hipLaunchKernelGGL(L.M <= 5 ? &k_control<5> : &k_control<kMaxDepth>, dim3(1),
                       dim3(kCtlThreads), 0, s, st, at<double>(ws, L.off_part),
                       (int)nblk, L.M, inv_count, op->tol, op->max_iter, (float)op->mdiis_eta,
                       op->eta_dynamic, (int)op->accelerator, op->anderson_s1, op->anderson_s2,
                       anchor ? 1 : 0, at<double2>(ws, L.off_hist), (size_t)0);
  }
}

int order_of(const rism3d_opts* op) { return op->closure == RISM3D_PSE ? op->pse_order : 1; }

// ---------------------------------------------------------------------------
// Graph cache: one instantiated graph per (workspace, problem shape, options,
// timing switch), holding one anchor period of iterations.  Kernel arguments
// depend only on these, so a graph is valid for every later solve with the
// same key.  Library-owned, host side; rism3d_release_graphs() frees it.
// ---------------------------------------------------------------------------
bool g_use_graphs = true;

struct GraphEntry {
  std::string key;
  hipGraphExec_t exec = nullptr;
  std::vector<Timer::Pending> timing;   // event pairs recorded inside the graph
  void harvest(int executed) {
    for (const Timer::Pending& p : timing) {
      float t = 0.0f;
      if (p.tag >= executed) continue;
      if (hipEventElapsedTime(&t, p.a, p.b) == hipSuccess) {
        g_timer.ms[p.fam] += t;
        g_timer.count[p.fam] += 1;
      } else {
        (void)hipGetLastError();
      }
    }
  }
};

std::mutex g_graph_mu;
std::vector<GraphEntry*> g_graphs;   // most recent last
constexpr size_t kMaxGraphs = 32;

// One capture stream per device (default priority, non-blocking), created on
// first use and kept for the life of the process.
hipStream_t capture_stream() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  static std::vector<hipStream_t> streams;
  if ((int)streams.size() <= dev) streams.resize(dev + 1, nullptr);
  if (!streams[dev] && hipStreamCreateWithFlags(&streams[dev], hipStreamNonBlocking) != hipSuccess) {
    (void)hipGetLastError();
    streams[dev] = nullptr;
  }
  return streams[dev];
}

std::string graph_key(const Layout& L, const void* ws, const rism3d_opts* op, double inv_dkt,
                      int every, Batch bt) {
  char buf[512];
  snprintf(buf, sizeof(buf),
           "%p|%zu|%d,%d,%d,%d,%d,%d|%d,%d,%.17g,%d,%.17g,%d,%d|%a|%d|%d,%zu|%d,%a,%a|%a,%a,%a",
           ws, L.total, L.nx, L.ny, L.nz, L.nv, L.M, L.m_tab, (int)op->closure, op->pse_order,
           op->tol, op->max_iter, op->mdiis_eta, op->eta_dynamic, every, inv_dkt,
           g_timer.on ? g_timer.only : -2, bt.nb, bt.stride, (int)op->accelerator,
           op->anderson_s1, op->anderson_s2, L.dkx, L.dky, L.dkz);
  std::string key = buf;
  for (int g = 0; g < kMaxSites; ++g) {   // Gram weights are kernel arguments too
    snprintf(buf, sizeof(buf), ",%a", (double)L.gw.w[g]);
    key += buf;
  }
  return key;
}

void drop_graph(GraphEntry* e) {
  if (e->exec) (void)hipGraphExecDestroy(e->exec);
  for (const Timer::Pending& p : e->timing) {
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  delete e;
}

GraphEntry* graph_for(const Layout& L, void* ws, const rism3d_opts* op, double inv_dkt, int every,
                      hipStream_t s, Batch bt = {}) {
  const std::string key = graph_key(L, ws, op, inv_dkt, every, bt);
  std::lock_guard<std::mutex> lock(g_graph_mu);
  for (size_t i = 0; i < g_graphs.size(); ++i) {
    if (g_graphs[i]->key == key) {
      GraphEntry* e = g_graphs[i];
      g_graphs.erase(g_graphs.begin() + i);
      g_graphs.push_back(e);
      return e;
    }
  }
  // Capture on a library-owned stream of the current device (the caller's
  // stream may be the null stream, which cannot be captured); the graph is
  // then launched on the caller's stream.  Anything recorded by the timer
  // during the capture belongs to the graph.
  hipStream_t cs = capture_stream();
  if (!cs) return nullptr;
  std::vector<Timer::Pending> before;
  before.swap(g_timer.pending);
  hipGraph_t graph = nullptr;
  if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    (void)hipGetLastError();
    g_timer.pending.swap(before);
    return nullptr;
  }
  g_capturing = true;
  g_capture_bad = false;
  for (int k = 0; k < every; ++k) {
    g_iter_tag = k;
    launch_iteration(L, ws, op, inv_dkt, k == 0, cs, bt);
  }
  g_iter_tag = -1;
  g_capturing = false;
  const hipError_t ec = hipStreamEndCapture(cs, &graph);
  GraphEntry* e = new GraphEntry;
  e->key = key;
  e->timing.swap(g_timer.pending);
  g_timer.pending.swap(before);
  if (ec != hipSuccess || !graph || g_capture_bad ||
      hipGraphInstantiate(&e->exec, graph, nullptr, nullptr, 0) != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    (void)hipGetLastError();
    drop_graph(e);
    return nullptr;
  }
  (void)hipGraphDestroy(graph);
  if (g_graphs.size() >= kMaxGraphs) {
    drop_graph(g_graphs.front());
    g_graphs.erase(g_graphs.begin());
  }
  g_graphs.push_back(e);
  return e;
}

// Potential, long-range spectrum, susceptibility and twiddle tables of one
// problem into its workspace (the work of rism3d_potential after validation).
rism3d_status prepare(const rism3d_problem* pr, const Layout& L, void* ws, hipStream_t s) {
  const double r0x = pr->center[0] - (pr->nx / 2) * pr->spacing;
  const double r0y = pr->center[1] - (pr->ny / 2) * pr->spacing;
  const double r0z = pr->center[2] - (pr->nz / 2) * pr->spacing;
  const SiteConsts sc = site_consts(pr, L.beta);
  SiteLJ sl;
  memset(&sl, 0, sizeof(sl));
  for (int g = 0; g < pr->n_sites; ++g) {
    sl.sigma[g] = pr->site_sigma[g];
    sl.eps[g] = pr->site_eps[g];
  }
  if (L.n_atoms > 0) {
    hipLaunchKernelGGL(k_prep_atoms, dim3(blocks_for(L.n_atoms, 256)), dim3(256), 0, s, pr->xyz,
                       pr->q, pr->sigma, pr->eps, L.n_atoms, r0x, r0y, r0z, L.beta, L.nv, sl,
                       at<double4>(ws, L.off_atoms), at<double2>(ws, L.off_lj));
    LAUNCH_CHECK();
    const int nsum = L.nx + L.ny + L.nz;
    hipLaunchKernelGGL(k_phase_tables, dim3(blocks_for((size_t)L.n_atoms * nsum, 256)), dim3(256),
                       0, s, pr->xyz, L.n_atoms, L.nx, L.ny, L.nz, r0x, r0y, r0z, L.dkx, L.dky,
                       L.dkz, at<double2>(ws, L.off_ph));
    LAUNCH_CHECK();
  }
  launch_potential(L, ws, pr->spacing, sc, s);
  LAUNCH_CHECK();
  const double pref = 4.0 * M_PI * L.beta * kCoulomb / (kScreen * kScreen) / L.dv;
  {
    TIMED(F_FTILDE, s);
    hipLaunchKernelGGL(k_ftilde, dim3(blocks_for(L.half, 256)), dim3(256), 0, s,
                       at<double2>(ws, L.off_ph), at<double4>(ws, L.off_atoms), L.n_atoms, L.nx, L.ny,
                       L.nz, L.dkx, L.dky, L.dkz, pref, at<double2>(ws, L.off_F));
  }
  LAUNCH_CHECK();
  hipLaunchKernelGGL(k_chi_tables, dim3(blocks_for((size_t)L.m_tab * L.nv, 256)), dim3(256), 0, s,
                     pr->chi, L.nv, pr->n_k, L.m_tab, 1.0 / (double)L.N, sc,
                     at<float>(ws, L.off_chi32), at<double>(ws, L.off_chi64),
                     at<double>(ws, L.off_q64));
  LAUNCH_CHECK();
  const int dims[3] = {L.nx, L.ny, L.nz};
  for (int a = 0; a < 3; ++a)
    hipLaunchKernelGGL(k_twiddles, dim3(blocks_for(2 * dims[a], 256)), dim3(256), 0, s, dims[a],
                       at<float2>(ws, L.off_tw32[a]), at<double2>(ws, L.off_tw64[a]));
  hipLaunchKernelGGL(k_mark_prepared, dim3(1), dim3(1), 0, s, at<IterState>(ws, L.off_state),
                     layout_key(L));
  LAUNCH_CHECK();
  return RISM3D_OK;
}

// Launches the SFE density sums of a solved workspace into its output slot
// (read back with read_sfe after the stream synchronises).
void launch_sfe(const rism3d_problem* pr, const rism3d_opts* op, const Layout& L, void* ws,
                hipStream_t s) {
  const SiteConsts sc = site_consts(pr, L.beta);
  unsigned nblk = blocks_for(L.N, kRedThreads);
  if (nblk > (unsigned)kRedBlocks) nblk = kRedBlocks;
  {
    TIMED(F_SFE, s);
    hipLaunchKernelGGL(k_sfe_partial, dim3(nblk), dim3(kRedThreads), 0, s,
                       at<IterState>(ws, L.off_state), at<float>(ws, L.off_tau),
                       at<float>(ws, L.off_tref), at<float>(ws, L.off_tlo), at<float>(ws, L.off_w),
                       at<float>(ws, L.off_phi), L.N, L.nv,
                       (int)op->closure, order_of(op), sc, at<double>(ws, L.off_part));
  }
  const double scale = L.dv / L.beta;   // k_B T dV
  hipLaunchKernelGGL(k_sfe_reduce, dim3(1), dim3(kRedThreads), 0, s, at<double>(ws, L.off_part),
                     (int)nblk, L.nv, scale, L.dv, sc, at<double>(ws, L.off_out));
}

// Host finish of the thermodynamics: Eq 19 (PMV) and Eq 21 (PC term) from the
// kernels' rho_g \int c_g and the bulk solvent's chi_T and pressure.
void fill_thermo(const double* res, const rism3d_problem* pr, rism3d_thermo_out* out) {
  memset(out, 0, sizeof(*out));
  out->sfe = res[kMaxSites];
  double sum_c = 0.0;
  for (int g = 0; g < pr->n_sites; ++g) {
    out->sfe_site[g] = res[g];
    out->rho_int_c[g] = res[kMaxSites + 1 + g];
    sum_c += out->rho_int_c[g];
  }
  out->rho_int_c_total = sum_c;
  if (pr->compressibility > 0.0) {
    out->pmv = kBoltzmann * pr->temperature * pr->compressibility * (1.0 - sum_c);
    out->pc = -pr->pressure * out->pmv;
  } else {
    out->pmv = out->pc = std::nan("");
  }
  out->sfe_pc = out->sfe + out->pc;
}

// ---------------------------------------------------------------------------
// Batched solves.  Members are grouped by the iteration layout (grid, sites,
// MDIIS depth, table length and spacing); a group whose axis lengths have the
// fixed-size fused kernels runs as one batched launch per kernel (blockIdx.y =
// member), other members as groups of one.  The batch workspace holds a state
// table (one IterState copy per member, gathered after each chunk) followed by
// the groups, member m of a group at off + m * stride.
// ---------------------------------------------------------------------------
struct BatchGroup {
  Layout L;                  // layout of the first member, total = the stride
  double inv_dkt = 0.0f;
  bool batched = false;
  size_t off = 0, stride = 0;
  std::vector<int> members;  // indices into the problem array
};

__global__ void k_gather_states(const char* __restrict__ base, size_t stride, size_t off_state,
                                const int* __restrict__ slots, IterState* __restrict__ table) {
  const int m = blockIdx.x;
  const int* src = reinterpret_cast<const int*>(base + (size_t)m * stride + off_state);
  int* dst = reinterpret_cast<int*>(table + slots[m]);
  for (int i = threadIdx.x; i < (int)(sizeof(IterState) / sizeof(int)); i += blockDim.x)
    dst[i] = src[i];
}

bool batchable(const Layout& L) {
  return fixed_fft_size(L.nx) && fixed_fft_size(L.ny) && zcz_supported(L);
}

bool same_iteration_layout(const Layout& a, const Layout& b) {
  return a.nx == b.nx && a.ny == b.ny && a.nz == b.nz && a.nv == b.nv && a.M == b.M &&
         a.m_tab == b.m_tab && a.off_out == b.off_out &&
         std::memcmp(a.gw.w, b.gw.w, sizeof(a.gw.w)) == 0;
}

struct BatchPlan {
  std::vector<BatchGroup> groups;
  size_t off_table = 0;   // IterState[n]: member states gathered after each chunk
  size_t off_index = 0;   // int[n]: problem index of each group member, group by group
  size_t total = 0;
};

rism3d_status batch_plan(int n, const rism3d_problem* prs, const rism3d_opts* op,
                         BatchPlan* plan) {
  std::vector<BatchGroup>* groups = &plan->groups;
  if (n < 1 || !prs || !op) return fail(RISM3D_E_ARG, "empty batch or null arguments");
  groups->clear();
  for (int i = 0; i < n; ++i) {
    Layout L;
    const rism3d_status st = make_layout(&prs[i], op, &L);
    if (st != RISM3D_OK)
      return fail(st, "batch member %d: %s", i, g_error.c_str());
    const double inv_dkt = (1.0 / prs[i].dk);
    BatchGroup* hit = nullptr;
    if (batchable(L))
      for (BatchGroup& g : *groups)
        if (g.batched && same_iteration_layout(g.L, L) && g.inv_dkt == inv_dkt &&
            prs[g.members[0]].spacing == prs[i].spacing) {
          hit = &g;
          break;
        }
    if (hit) {
      hit->members.push_back(i);
      if (L.total > hit->L.total) hit->L.total = L.total;
    } else {
      BatchGroup g;
      g.L = L;
      g.inv_dkt = inv_dkt;
      g.batched = batchable(L);
      g.members.push_back(i);
      groups->push_back(g);
    }
  }
  size_t off = 0;
  plan->off_table = off;
  off = align_up(off + (size_t)n * sizeof(IterState));
  plan->off_index = off;
  off = align_up(off + (size_t)n * sizeof(int));
  for (BatchGroup& g : *groups) {
    g.stride = align_up(g.L.total);
    g.off = off;
    off += g.stride * g.members.size();
  }
  plan->total = off;
  return RISM3D_OK;
}

// ---------------------------------------------------------------------------
// Warm start: network input and training target from a solver workspace, and
// the Ornstein-Zernike half-step that turns a predicted c_sr into tau0.
// ---------------------------------------------------------------------------
#include "unet_host.hpp"

// x[g][n] = symlog(beta u_g(n)) with the capped beta u = w + f, f_g = beta C q_g phi.
__global__ void k_net_input(const float* __restrict__ w, const float* __restrict__ phi, size_t N,
                            int nv, SiteConsts sc, float* __restrict__ x) {
  const size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= (size_t)nv * N) return;
  const int g = (int)(id / N);
  const double bu = (double)w[id] + sc.coul64[g] * (double)phi[id - (size_t)g * N];
  x[id] = (float)(bu < 0.0 ? -log1p(-bu) : log1p(bu));
}

// c_sr = g - 1 - tau of the accepted iterate (FP64 closure).
__global__ void k_csr_out(const IterState* __restrict__ st, const float* __restrict__ tau_hist,
                          const float* __restrict__ tau_ref, const float* __restrict__ tau_lo,
                          const float* __restrict__ w, size_t N, int nv, int kind, int order,
                          float* __restrict__ c) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)nv * N) return;
  const int slot = st->final_slot;
  if (slot < 0) return;
  const double tau = ((double)tau_ref[idx] + (double)tau_lo[idx]) +
                     (double)tau_hist[(size_t)slot * nv * N + idx];
  c[idx] = (float)(closure_g(-(double)w[idx] + tau, kind, order) - 1.0 - tau);
}

// Packed FP64 pairs of the scaled prediction: spec[p][n] = s (c_{2p} + i c_{2p+1}).
__global__ void k_pack_c64(const float* __restrict__ c, size_t N, int nv, double scale,
                           double2* __restrict__ spec) {
  const size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int np = (nv + 1) / 2;
  if (id >= (size_t)np * N) return;
  const int p = (int)(id / N);
  const size_t n = id - (size_t)p * N;
  const double re = scale * (double)c[(size_t)(2 * p) * N + n];
  const double im = 2 * p + 1 < nv ? scale * (double)c[(size_t)(2 * p + 1) * N + n] : 0.0;
  spec[id] = make_double2(re, im);
}

// tau0 = h - c0 with h unpacked from the inverse-transformed pairs.
__global__ void k_tau_from_h(const double2* __restrict__ spec, const float* __restrict__ c,
                             size_t N, int nv, double scale, float* __restrict__ tau0) {
  const size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= (size_t)nv * N) return;
  const int g = (int)(id / N);
  const size_t n = id - (size_t)g * N;
  const double2 h = spec[(size_t)(g / 2) * N + n];
  tau0[id] = (float)(((g & 1) ? h.y : h.x) - scale * (double)c[id]);
}

// A state with every MDIIS slot stored and equal coefficients, so that timed
// launches of the fused kernels do the work of a steady-state iteration.
__global__ void k_tune_state(IterState* st, int M, float eta) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  for (int i = 0; i < kMaxDepth; ++i) {
    st->stored[i] = i < M;
    st->coef[i] = i < M ? 1.0f / (float)M : 0.0f;
    st->stamp[i] = i;
  }
  st->eta = eta;
  st->dest = 0;
  st->newest = M - 1;
  st->iter = 1;
  st->done = 0;
  st->converged = 0;
  st->status = 0;
  st->final_slot = -1;
  st->hold = 0;
}

template <int NV>
void launch_sfe_grad_nv(const Layout& L, const void* ws, const float* g, double dr,
                        const SiteConsts& sc, double scale, unsigned nb, double* dst,
                        hipStream_t s) {
  const dim3 grid(nb, (unsigned)((L.n_atoms + kGradAtoms - 1) / kGradAtoms));
  TIMED(F_SFEGRAD, s);
  hipLaunchKernelGGL(k_sfe_grad<NV>, grid, dim3(kGradThreads), 0, s,
                     at<double4>(const_cast<void*>(ws), L.off_atoms),
                     at<double2>(const_cast<void*>(ws), L.off_lj), L.n_atoms, g, L.nx, L.ny, L.N,
                     dr, sc, dst, scale);
}

// The shifted 3D transform of rism3d_transform with its twiddle tables in ws
// (rism3d_transform_workspace_bytes(nx, ny, nz) bytes, 256-byte aligned).
rism3d_status transform_on(int nx, int ny, int nz, int count, void* d_data, int forward, void* ws,
                           hipStream_t s) {
  Layout L;
  memset(&L, 0, sizeof(L));
  plan_axis(nx, &L.px);
  plan_axis(ny, &L.py);
  plan_axis(nz, &L.pz);
  L.nx = nx;
  L.ny = ny;
  L.nz = nz;
  L.npair = count;
  L.N = (size_t)nx * ny * nz;
  const size_t offs[3] = {0, align_up(2 * (size_t)nx * sizeof(float2)),
                          align_up(2 * (size_t)nx * sizeof(float2)) +
                              align_up(2 * (size_t)ny * sizeof(float2))};
  const int dims[3] = {nx, ny, nz};
  const float2* tw[3];
  for (int a = 0; a < 3; ++a) {
    hipLaunchKernelGGL(k_twiddles, dim3(blocks_for(2 * dims[a], 256)), dim3(256), 0, s, dims[a],
                       at<float2>(ws, offs[a]), (double2*)nullptr);
    tw[a] = at<float2>(ws, offs[a]);
  }
  launch_fft3_on(L, static_cast<float2*>(d_data), tw, forward, (const int*)nullptr, s);
  LAUNCH_CHECK();
  return RISM3D_OK;
}

// Address of the file-scope scratch array on the current device, looked up
// once per device (hipGetSymbolAddress) and kept: the array's name in host
// code is not a device address.
std::mutex g_scratch_mu;
constexpr int kMaxDevices = 64;
void* g_scratch_dev[kMaxDevices] = {};

rism3d_status scratch_address(void** out) {
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(RISM3D_E_DEVICE, "device index %d", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(RISM3D_E_DEVICE, "hipGetSymbolAddress(scratch) failed: %s",
                  hipGetErrorString(e));
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  return RISM3D_OK;
}

}  // namespace

extern "C" {

void rism3d_use_graphs(int on) { g_use_graphs = on != 0; }

void rism3d_release_graphs(void) {
  std::lock_guard<std::mutex> lock(g_graph_mu);
  for (GraphEntry* e : g_graphs) drop_graph(e);
  g_graphs.clear();
}

size_t rism3d_workspace_bytes(const rism3d_problem* problem, const rism3d_opts* opts) {
  Layout L;
  if (make_layout(problem, opts, &L) != RISM3D_OK) return 0;
  return L.total;
}

rism3d_status rism3d_potential(const rism3d_problem* pr, const rism3d_opts* op, void* ws,
                               size_t ws_bytes, hipStream_t s) {
  Layout L;
  rism3d_status st = make_layout(pr, op, &L);
  if (st != RISM3D_OK) return st;
  if ((st = check_ws(L, ws, ws_bytes)) != RISM3D_OK) return st;
  return prepare(pr, L, ws, s);
}


rism3d_status rism3d_solve(const rism3d_problem* pr, const rism3d_opts* op, const float* tau0,
                           void* ws, size_t ws_bytes, float* g_out, rism3d_info* info,
                           hipStream_t s) {
  Layout L;
  rism3d_status st = make_layout(pr, op, &L);
  if (st != RISM3D_OK) return st;
  if ((st = check_ws(L, ws, ws_bytes)) != RISM3D_OK) return st;
  IterState* dst = at<IterState>(ws, L.off_state);
  IterState host;
  HIP_TRY(hipMemcpyAsync(&host, dst, sizeof(IterState), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if ((st = check_prepared(host, L)) != RISM3D_OK) return st;
  const double inv_dkt = (1.0 / pr->dk);
  // A caller's starting tau is only a starting point: if the iteration from
  // it ends on a non-finite residual, the solve is repeated from tau0 = 0.
  for (int attempt = 0; attempt < 2; ++attempt) {
  const float* t0 = attempt == 0 ? tau0 : nullptr;
  hipLaunchKernelGGL(k_init_state, dim3(1), dim3(1), 0, s, dst, (float)op->mdiis_eta,
                     t0 ? 1 : 0);
  hipLaunchKernelGGL(k_init_tau, dim3(blocks_for((size_t)L.nv * L.N, kElemThreads)),
                     dim3(kElemThreads), 0, s, t0, at<float>(ws, L.off_tau),
                     at<float>(ws, L.off_tref), at<float>(ws, L.off_tlo),
                     (size_t)L.nv * L.N);
  LAUNCH_CHECK();
  const int every = op->anchor_every > 0 ? op->anchor_every : kDefaultAnchorEvery;
  // One anchor period (an FP64 anchor evaluation + every-1 FP32 increments) is
  // captured once into a HIP graph per workspace and options, then replayed;
  // the host reads the small device state after each replay.
  GraphEntry* graph = g_use_graphs ? graph_for(L, ws, op, inv_dkt, every, s) : nullptr;
  const int chunk = graph ? every : (op->check_every > 0 ? op->check_every : kDefaultCheckEvery);
  int launched = 0;
  int iter_before = 0;
  int phase = 0;   // direct launches: iterations since the last FP64 anchor
  for (;;) {
    if (graph) {
      HIP_TRY(hipGraphLaunch(graph->exec, s));   // an anchor period starts with the anchor
      launched += every;
    } else {
      int todo = (op->max_iter - launched) < chunk ? (op->max_iter - launched) : chunk;
      if (todo < 1) todo = 1;   // past max_iter only while a verification is pending
      for (int k = 0; k < todo; ++k) {
        g_iter_tag = k;
        launch_iteration(L, ws, op, inv_dkt, phase == 0, s);
        phase = (phase + 1) % every;
      }
      g_iter_tag = -1;
      launched += todo;
    }
    LAUNCH_CHECK();
    HIP_TRY(hipMemcpyAsync(&host, dst, sizeof(IterState), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (g_timer.on) {
      const int executed = host.iter - iter_before;
      if (graph) graph->harvest(executed);
      g_timer.harvest(executed);
    }
    iter_before = host.iter;
    if (host.done == kDoneFinished) break;
    // An FP32 residual passed the tolerance: the next FP64 evaluation decides
    // (every evaluation counts towards max_iter, so this ends).
    if (host.done == kDoneVerify) {
      phase = 0;
      continue;
    }
    if (launched >= op->max_iter) break;
  }
  if (!(t0 && host.status == RISM3D_E_NONFINITE)) break;
  }
  if (g_out) {
    hipLaunchKernelGGL(k_output, dim3(blocks_for((size_t)L.nv * L.N, kElemThreads)),
                       dim3(kElemThreads), 0, s, dst, at<float>(ws, L.off_tau),
                       at<float>(ws, L.off_tref), at<float>(ws, L.off_tlo),
                       at<float>(ws, L.off_w), L.N, L.nv,
                       (int)op->closure, order_of(op), g_out, (float*)nullptr);
    LAUNCH_CHECK();
  }
  if (info) {
    info->iterations = host.iter;
    info->rms = host.last_rms;
    info->restarts = host.restarts;
    info->warm_start_used = host.warm;
  }
  if (host.done != kDoneFinished)
    return fail(RISM3D_E_NOCONV, "no convergence in %d iterations", host.iter);
  if (host.status == RISM3D_E_NONFINITE)
    return fail(RISM3D_E_NONFINITE, "non-finite residual at iteration %d", host.iter);
  if (host.status == RISM3D_E_NOCONV)
    return fail(RISM3D_E_NOCONV, "rms %g above tol %g after %d iterations", host.last_rms,
                op->tol, host.iter);
  g_error.clear();
  return RISM3D_OK;
}

rism3d_status rism3d_solve_ladder(const rism3d_problem* pr, const rism3d_opts* stages,
                                  int n_stages, const float* tau0, void* ws, size_t ws_bytes,
                                  float* g_out, rism3d_info* info, hipStream_t s) {
  if (n_stages < 1 || !stages) return fail(RISM3D_E_ARG, "n_stages must be >= 1");
  Layout L0;
  rism3d_status st = make_layout(pr, &stages[0], &L0);
  if (st != RISM3D_OK) return st;
  const unsigned key = layout_key(L0);
  for (int k = 1; k < n_stages; ++k) {
    Layout Lk;
    if ((st = make_layout(pr, &stages[k], &Lk)) != RISM3D_OK) return st;
    if (layout_key(Lk) != key)
      return fail(RISM3D_E_ARG,
                  "ladder stage %d changes the workspace layout (MDIIS depth or accelerator)", k);
  }
  // Between stages the returned iterate, rounded to float32, is the next
  // start; it is staged in the closure-increment section, which the first
  // kernel of a solve reads before any kernel writes it.
  float* start = at<float>(ws, L0.off_dg);
  for (int k = 0; k < n_stages; ++k) {
    const rism3d_opts* op = &stages[k];
    const float* t0 = tau0;
    if (k > 0) {
      hipLaunchKernelGGL(k_output, dim3(blocks_for((size_t)L0.nv * L0.N, kElemThreads)),
                         dim3(kElemThreads), 0, s, at<IterState>(ws, L0.off_state),
                         at<float>(ws, L0.off_tau), at<float>(ws, L0.off_tref),
                         at<float>(ws, L0.off_tlo), at<float>(ws, L0.off_w), L0.N, L0.nv,
                         (int)op->closure, order_of(op), (float*)nullptr, start);
      LAUNCH_CHECK();
      t0 = start;
    }
    st = rism3d_solve(pr, op, t0, ws, ws_bytes, k + 1 == n_stages ? g_out : nullptr,
                      info ? &info[k] : nullptr, s);
    // a stage short of its tolerance still hands its iterate on; the last
    // stage's status is the ladder's
    if (st != RISM3D_OK && !(st == RISM3D_E_NOCONV && k + 1 < n_stages)) return st;
  }
  return RISM3D_OK;
}

rism3d_status rism3d_thermo(const rism3d_problem* pr, const rism3d_opts* op, const void* ws_c,
                            size_t ws_bytes, rism3d_thermo_out* out, hipStream_t s) {
  Layout L;
  rism3d_status st = make_layout(pr, op, &L);
  if (st != RISM3D_OK) return st;
  if ((st = check_ws(L, ws_c, ws_bytes)) != RISM3D_OK) return st;
  if (!out) return fail(RISM3D_E_ARG, "null output");
  void* ws = const_cast<void*>(ws_c);
  IterState* dst = at<IterState>(ws, L.off_state);
  IterState host;
  HIP_TRY(hipMemcpyAsync(&host, dst, sizeof(IterState), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if ((st = check_prepared(host, L)) != RISM3D_OK) return st;
  if (host.final_slot < 0)
    return fail(RISM3D_E_WORKSPACE, "no solution in the workspace: call rism3d_solve first");
  launch_sfe(pr, op, L, ws, s);
  LAUNCH_CHECK();
  double res[kOutDoubles];
  HIP_TRY(hipMemcpyAsync(res, at<double>(ws, L.off_out), sizeof(res), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (g_timer.on) g_timer.harvest();
  fill_thermo(res, pr, out);
  g_error.clear();
  return RISM3D_OK;
}

rism3d_status rism3d_sfe_gradient(const rism3d_problem* pr, const rism3d_opts* op, const float* g,
                                  void* ws, size_t ws_bytes, double* grad, hipStream_t s) {
  Layout L;
  rism3d_status st = make_layout(pr, op, &L);
  if (st != RISM3D_OK) return st;
  if ((st = check_ws(L, ws, ws_bytes)) != RISM3D_OK) return st;
  if (!g) return fail(RISM3D_E_ARG, "null g");
  if (L.n_atoms > 0 && !grad) return fail(RISM3D_E_ARG, "null gradient output");
  IterState host;
  HIP_TRY(hipMemcpyAsync(&host, at<IterState>(ws, L.off_state), sizeof(IterState),
                         hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if ((st = check_prepared(host, L)) != RISM3D_OK) return st;
  if (L.n_atoms == 0) {
    g_error.clear();
    return RISM3D_OK;
  }
  // One partial row of 3 n_atoms doubles per workgroup column, kept in the
  // spectrum section (scratch between iterations).  About 2048 workgroups in
  // all; a single column writes the result directly.
  const size_t tiles = (L.N + kGradTile - 1) / kGradTile;
  const size_t chunks = (L.n_atoms + kGradAtoms - 1) / kGradAtoms;
  size_t nb = std::max<size_t>(1, 2048 / chunks);
  nb = std::min(nb, tiles);
  const size_t row = (size_t)L.n_atoms * 3 * sizeof(double);
  nb = std::min(nb, (size_t)L.npair * L.N * sizeof(double2) / row);
  if (nb < 1) nb = 1;
  const SiteConsts sc = site_consts(pr, L.beta);
  const double scale = L.dv / L.beta;   // k_B T dV
  double* dst = nb == 1 ? grad : at<double>(ws, L.off_spec);
  switch (L.nv) {
    case 1: launch_sfe_grad_nv<1>(L, ws, g, pr->spacing, sc, scale, (unsigned)nb, dst, s); break;
    case 2: launch_sfe_grad_nv<2>(L, ws, g, pr->spacing, sc, scale, (unsigned)nb, dst, s); break;
    case 3: launch_sfe_grad_nv<3>(L, ws, g, pr->spacing, sc, scale, (unsigned)nb, dst, s); break;
    case 4: launch_sfe_grad_nv<4>(L, ws, g, pr->spacing, sc, scale, (unsigned)nb, dst, s); break;
    case 5: launch_sfe_grad_nv<5>(L, ws, g, pr->spacing, sc, scale, (unsigned)nb, dst, s); break;
    case 6: launch_sfe_grad_nv<6>(L, ws, g, pr->spacing, sc, scale, (unsigned)nb, dst, s); break;
    case 7: launch_sfe_grad_nv<7>(L, ws, g, pr->spacing, sc, scale, (unsigned)nb, dst, s); break;
    default: launch_sfe_grad_nv<8>(L, ws, g, pr->spacing, sc, scale, (unsigned)nb, dst, s); break;
  }
  LAUNCH_CHECK();
  if (nb > 1) {
    const int n3 = L.n_atoms * 3;
    hipLaunchKernelGGL(k_sfe_grad_reduce, dim3(blocks_for(n3, 256)), dim3(256), 0, s, dst, (int)nb,
                       n3, grad);
    LAUNCH_CHECK();
  }
  if (g_timer.on) {
    HIP_TRY(hipStreamSynchronize(s));
    g_timer.harvest();
  }
  g_error.clear();
  return RISM3D_OK;
}

size_t rism3d_batch_workspace_bytes(int n, const rism3d_problem* problems,
                                    const rism3d_opts* opts) {
  BatchPlan plan;
  if (batch_plan(n, problems, opts, &plan) != RISM3D_OK) return 0;
  return plan.total;
}

rism3d_status rism3d_solve_batch(int n, const rism3d_problem* prs, const rism3d_opts* op,
                                 const float* const* tau0, void* ws, size_t ws_bytes,
                                 float* const* g_out, rism3d_info* info,
                                 rism3d_thermo_out* thermo, hipStream_t s) {
  BatchPlan plan;
  rism3d_status st = batch_plan(n, prs, op, &plan);
  if (st != RISM3D_OK) return st;
  if (!ws) return fail(RISM3D_E_WORKSPACE, "null workspace");
  if (((uintptr_t)ws) & 255) return fail(RISM3D_E_WORKSPACE, "workspace must be 256-byte aligned");
  if (ws_bytes < plan.total)
    return fail(RISM3D_E_WORKSPACE, "batch workspace holds %zu bytes, %zu needed", ws_bytes,
                plan.total);
  char* base = static_cast<char*>(ws);
  auto member_ws = [&](const BatchGroup& g, size_t m) -> void* {
    return base + g.off + m * g.stride;
  };
  // problem index of each group member, group by group
  std::vector<int> index;
  for (const BatchGroup& g : plan.groups) index.insert(index.end(), g.members.begin(), g.members.end());
  HIP_TRY(hipMemcpyAsync(base + plan.off_index, index.data(), index.size() * sizeof(int),
                         hipMemcpyHostToDevice, s));
  // set-up and start of every member
  for (const BatchGroup& g : plan.groups)
    for (size_t m = 0; m < g.members.size(); ++m) {
      const int i = g.members[m];
      Layout L;
      make_layout(&prs[i], op, &L);
      void* w = member_ws(g, m);
      if ((st = prepare(&prs[i], L, w, s)) != RISM3D_OK)
        return fail(st, "batch member %d: %s", i, g_error.c_str());
      const float* t0 = tau0 ? tau0[i] : nullptr;
      hipLaunchKernelGGL(k_init_state, dim3(1), dim3(1), 0, s, at<IterState>(w, L.off_state),
                         (float)op->mdiis_eta, t0 ? 1 : 0);
      hipLaunchKernelGGL(k_init_tau, dim3(blocks_for((size_t)L.nv * L.N, kElemThreads)),
                         dim3(kElemThreads), 0, s, t0, at<float>(w, L.off_tau),
                         at<float>(w, L.off_tref), at<float>(w, L.off_tlo),
                         (size_t)L.nv * L.N);
      LAUNCH_CHECK();
    }
  const int every = op->anchor_every > 0 ? op->anchor_every : kDefaultAnchorEvery;
  const size_t ng = plan.groups.size();
  std::vector<GraphEntry*> graphs(ng, nullptr);
  std::vector<Batch> batches(ng);
  for (size_t k = 0; k < ng; ++k) {
    const BatchGroup& g = plan.groups[k];
    batches[k] = Batch{(int)g.members.size(), g.batched ? g.stride : 0};
    if (g_use_graphs)
      graphs[k] = graph_for(g.L, member_ws(g, 0), op, g.inv_dkt, every, s, batches[k]);
  }
  const int chunk_direct = op->check_every > 0 ? op->check_every : kDefaultCheckEvery;
  std::vector<int> launched(ng, 0), iter_before(n, 0), phase(ng, 0);
  std::vector<char> finished(ng, 0);
  std::vector<IterState> host(n);
  IterState* table = at<IterState>(ws, plan.off_table);
  const int* index_d = at<int>(ws, plan.off_index);
  for (;;) {
    size_t first = 0;
    for (size_t k = 0; k < ng; ++k) {
      const BatchGroup& g = plan.groups[k];
      if (!finished[k]) {
        if (graphs[k]) {
          HIP_TRY(hipGraphLaunch(graphs[k]->exec, s));
          launched[k] += every;
        } else {
          const int left = op->max_iter - launched[k];
          int todo = left < chunk_direct ? left : chunk_direct;
          if (todo < 1) todo = 1;   // past max_iter only while a verification is pending
          for (int j = 0; j < todo; ++j) {
            g_iter_tag = j;
            launch_iteration(g.L, member_ws(g, 0), op, g.inv_dkt, phase[k] == 0, s, batches[k]);
            phase[k] = (phase[k] + 1) % every;
          }
          g_iter_tag = -1;
          launched[k] += todo;
        }
        hipLaunchKernelGGL(k_gather_states, dim3((unsigned)g.members.size()), dim3(64), 0, s,
                           static_cast<const char*>(member_ws(g, 0)), g.stride, g.L.off_state,
                           index_d + first, table);
      }
      first += g.members.size();
    }
    LAUNCH_CHECK();
    HIP_TRY(hipMemcpyAsync(host.data(), table, (size_t)n * sizeof(IterState),
                           hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    bool all = true;
    for (size_t k = 0; k < ng; ++k) {
      if (finished[k]) continue;
      const BatchGroup& g = plan.groups[k];
      bool done = true, verify = false;
      int executed = 0;
      for (int i : g.members) {
        done = done && host[i].done == kDoneFinished;
        verify = verify || host[i].done == kDoneVerify;
        executed = std::max(executed, host[i].iter - iter_before[i]);
        iter_before[i] = host[i].iter;
      }
      if (g_timer.on && graphs[k]) graphs[k]->harvest(executed);
      // a member whose FP32 residual passed waits for the next FP64 evaluation
      // (the start of an anchor period), also past max_iter
      if (verify) phase[k] = 0;
      if (done || (launched[k] >= op->max_iter && !verify)) finished[k] = 1;
      all = all && finished[k];
    }
    if (g_timer.on) g_timer.harvest();
    if (all) break;
  }
  // outputs, SFE and per-member status
  rism3d_status worst = RISM3D_OK;
  int worst_member = -1;
  std::vector<double> sfe((size_t)n * kOutDoubles, 0.0);
  for (const BatchGroup& g : plan.groups)
    for (size_t m = 0; m < g.members.size(); ++m) {
      const int i = g.members[m];
      Layout L;
      make_layout(&prs[i], op, &L);
      void* w = member_ws(g, m);
      const IterState& h = host[i];
      if (g_out && g_out[i])
        hipLaunchKernelGGL(k_output, dim3(blocks_for((size_t)L.nv * L.N, kElemThreads)),
                           dim3(kElemThreads), 0, s, at<IterState>(w, L.off_state),
                           at<float>(w, L.off_tau), at<float>(w, L.off_tref),
                           at<float>(w, L.off_tlo),
                           at<float>(w, L.off_w), L.N, L.nv, (int)op->closure, order_of(op),
                           g_out[i], (float*)nullptr);
      if (thermo && h.final_slot >= 0) {
        launch_sfe(&prs[i], op, L, w, s);
        HIP_TRY(hipMemcpyAsync(&sfe[(size_t)i * kOutDoubles], at<double>(w, L.off_out),
                               kOutDoubles * sizeof(double), hipMemcpyDeviceToHost, s));
      }
      LAUNCH_CHECK();
      rism3d_status ms = RISM3D_OK;
      if (h.done != kDoneFinished || h.status == RISM3D_E_NOCONV) ms = RISM3D_E_NOCONV;
      if (h.status == RISM3D_E_NONFINITE) ms = RISM3D_E_NONFINITE;
      if (info) {
        info[i].iterations = h.iter;
        info[i].rms = h.last_rms;
        info[i].restarts = h.restarts;
        info[i].warm_start_used = h.warm;
      }
      if (ms != RISM3D_OK && (worst == RISM3D_OK || ms == RISM3D_E_NONFINITE)) {
        worst = ms;
        worst_member = i;
      }
    }
  HIP_TRY(hipStreamSynchronize(s));
  if (g_timer.on) g_timer.harvest();
  if (thermo)
    for (int i = 0; i < n; ++i) {
      if (host[i].final_slot >= 0) fill_thermo(&sfe[(size_t)i * kOutDoubles], &prs[i], &thermo[i]);
      else memset(&thermo[i], 0, sizeof(thermo[i]));
    }
  if (worst != RISM3D_OK)
    return fail(worst, "batch member %d: %s after %d iterations (rms %g)", worst_member,
                worst == RISM3D_E_NONFINITE ? "non-finite residual" : "no convergence",
                host[worst_member].iter, host[worst_member].last_rms);
  g_error.clear();
  return RISM3D_OK;
}

rism3d_status rism3d_get_tau(const rism3d_problem* pr, const rism3d_opts* op, const void* ws_c,
                             size_t ws_bytes, float* d_tau, hipStream_t s) {
  Layout L;
  rism3d_status st = make_layout(pr, op, &L);
  if (st != RISM3D_OK) return st;
  if ((st = check_ws(L, ws_c, ws_bytes)) != RISM3D_OK) return st;
  if (!d_tau) return fail(RISM3D_E_ARG, "null output");
  void* ws = const_cast<void*>(ws_c);
  hipLaunchKernelGGL(k_output, dim3(blocks_for((size_t)L.nv * L.N, kElemThreads)),
                     dim3(kElemThreads), 0, s, at<IterState>(ws, L.off_state),
                     at<float>(ws, L.off_tau), at<float>(ws, L.off_tref),
                     at<float>(ws, L.off_tlo), at<float>(ws, L.off_w),
                     L.N, L.nv, (int)op->closure, order_of(op), (float*)nullptr, d_tau);
  LAUNCH_CHECK();
  return RISM3D_OK;
}

rism3d_status rism3d_get_history(const rism3d_problem* pr, const rism3d_opts* op,
                                 const void* ws_c, size_t ws_bytes, int capacity, double* rms,
                                 int* exact, int* count, hipStream_t s) {
  Layout L;
  rism3d_status st = make_layout(pr, op, &L);
  if (st != RISM3D_OK) return st;
  if ((st = check_ws(L, ws_c, ws_bytes)) != RISM3D_OK) return st;
  if (!count || capacity < 0 || (capacity > 0 && (!rms || !exact)))
    return fail(RISM3D_E_ARG, "null count, or null rms/exact with capacity > 0");
  void* ws = const_cast<void*>(ws_c);
  IterState host;
  HIP_TRY(hipMemcpyAsync(&host, at<IterState>(ws, L.off_state), sizeof(IterState),
                         hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if ((st = check_prepared(host, L)) != RISM3D_OK) return st;
  const int n = host.iter < kHistLen ? (host.iter > 0 ? host.iter : 0) : kHistLen;
  *count = n;
  const int take_n = n < capacity ? n : capacity;
  if (take_n > 0) {
    std::vector<double2> buf((size_t)take_n);
    HIP_TRY(hipMemcpyAsync(buf.data(), at<double2>(ws, L.off_hist),
                           (size_t)take_n * sizeof(double2), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    for (int i = 0; i < take_n; ++i) {
      rms[i] = buf[i].x;
      exact[i] = buf[i].y != 0.0;
    }
  }
  return RISM3D_OK;
}

rism3d_status rism3d_map(const rism3d_problem* pr, const rism3d_opts* op, const float* d_tau,
                         void* ws, size_t ws_bytes, float* d_res, double* rms, hipStream_t s) {
  Layout L;
  rism3d_status st = make_layout(pr, op, &L);
  if (st != RISM3D_OK) return st;
  if ((st = check_ws(L, ws, ws_bytes)) != RISM3D_OK) return st;
  if (!d_res) return fail(RISM3D_E_ARG, "null residual");
  IterState* dst = at<IterState>(ws, L.off_state);
  IterState host;
  HIP_TRY(hipMemcpyAsync(&host, dst, sizeof(IterState), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if ((st = check_prepared(host, L)) != RISM3D_OK) return st;
  if (!d_tau && host.final_slot < 0)
    return fail(RISM3D_E_WORKSPACE, "no solution in the workspace: call rism3d_solve first");
  rism3d_opts one = *op;
  one.max_iter = 1;
  one.tol = 0.0;   // never "converged": the single evaluation always runs to the end
  if (d_tau) {
    hipLaunchKernelGGL(k_init_state, dim3(1), dim3(1), 0, s, dst, (float)op->mdiis_eta, 1);
    hipLaunchKernelGGL(k_init_tau, dim3(blocks_for((size_t)L.nv * L.N, kElemThreads)),
                       dim3(kElemThreads), 0, s, d_tau, at<float>(ws, L.off_tau),
                       at<float>(ws, L.off_tref), at<float>(ws, L.off_tlo),
                       (size_t)L.nv * L.N);
  } else {
    // the held iterate; its evaluation re-bases the reference on that same
    // iterate, so the solution stays in place for rism3d_thermo and the outputs
    hipLaunchKernelGGL(k_hold_final, dim3(1), dim3(1), 0, s, dst);
  }
  launch_iteration(L, ws, &one, (1.0 / pr->dk), true, s);
  const size_t n = (size_t)L.nv * L.N;
  hipLaunchKernelGGL(k_copy_final_slot, dim3(blocks_for(n, kElemThreads)), dim3(kElemThreads), 0,
                     s, dst, at<float>(ws, L.off_res), d_res, n);
  LAUNCH_CHECK();
  HIP_TRY(hipMemcpyAsync(&host, dst, sizeof(IterState), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (rms) *rms = host.last_rms;
  g_error.clear();
  return RISM3D_OK;
}

rism3d_status rism3d_map_increment(const rism3d_problem* pr, const rism3d_opts* op,
                                   const float* d_tau_ref, const float* d_delta, void* ws,
                                   size_t ws_bytes, float* d_res, double* rms, hipStream_t s) {
  Layout L;
  rism3d_status st = make_layout(pr, op, &L);
  if (st != RISM3D_OK) return st;
  if ((st = check_ws(L, ws, ws_bytes)) != RISM3D_OK) return st;
  if (!d_tau_ref || !d_delta || !d_res) return fail(RISM3D_E_ARG, "null tau_ref, delta or residual");
  IterState* dst = at<IterState>(ws, L.off_state);
  IterState host;
  HIP_TRY(hipMemcpyAsync(&host, dst, sizeof(IterState), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if ((st = check_prepared(host, L)) != RISM3D_OK) return st;
  rism3d_opts two = *op;
  two.max_iter = 3;   // neither evaluation may end the iteration
  two.tol = 0.0;
  const size_t n = (size_t)L.nv * L.N;
  const double inv_dkt = 1.0 / pr->dk;
  hipLaunchKernelGGL(k_init_state, dim3(1), dim3(1), 0, s, dst, (float)op->mdiis_eta, 1);
  hipLaunchKernelGGL(k_init_tau, dim3(blocks_for(n, kElemThreads)), dim3(kElemThreads), 0, s,
                     d_tau_ref, at<float>(ws, L.off_tau), at<float>(ws, L.off_tref),
                     at<float>(ws, L.off_tlo), n);
  launch_iteration(L, ws, &two, inv_dkt, true, s);    // FP64: R_ref at tau_ref
  hipLaunchKernelGGL(k_set_increment, dim3(blocks_for(n, kElemThreads)), dim3(kElemThreads), 0, s,
                     dst, at<float>(ws, L.off_tau), d_delta, n);
  launch_iteration(L, ws, &two, inv_dkt, false, s);   // FP32: R_ref + dh - dg
  hipLaunchKernelGGL(k_copy_final_slot, dim3(blocks_for(n, kElemThreads)), dim3(kElemThreads), 0,
                     s, dst, at<float>(ws, L.off_res), d_res, n);
  LAUNCH_CHECK();
  HIP_TRY(hipMemcpyAsync(&host, dst, sizeof(IterState), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (rms) *rms = host.last_rms;
  g_error.clear();
  return RISM3D_OK;
}

rism3d_status rism3d_get_potential(const rism3d_problem* pr, const rism3d_opts* op,
                                   const void* ws_c, size_t ws_bytes, float* d_w, float* d_phi,
                                   hipStream_t s) {
  Layout L;
  rism3d_status st = make_layout(pr, op, &L);
  if (st != RISM3D_OK) return st;
  if ((st = check_ws(L, ws_c, ws_bytes)) != RISM3D_OK) return st;
  if (d_w)
    HIP_TRY(hipMemcpyAsync(d_w, at<float>(ws_c, L.off_w), (size_t)L.nv * L.N * sizeof(float),
                           hipMemcpyDeviceToDevice, s));
  if (d_phi)
    HIP_TRY(hipMemcpyAsync(d_phi, at<float>(ws_c, L.off_phi), L.N * sizeof(float),
                           hipMemcpyDeviceToDevice, s));
  return RISM3D_OK;
}

size_t rism3d_transform_workspace_bytes(int nx, int ny, int nz) {
  AxisPlan p;
  if (!plan_axis(nx, &p) || !plan_axis(ny, &p) || !plan_axis(nz, &p)) {
    fail(RISM3D_E_ARG, "grid %dx%dx%d unsupported", nx, ny, nz);
    return 0;
  }
  return align_up(2 * (size_t)nx * sizeof(float2)) + align_up(2 * (size_t)ny * sizeof(float2)) +
         align_up(2 * (size_t)nz * sizeof(float2));
}

rism3d_status rism3d_transform(int nx, int ny, int nz, int count, void* d_data, int forward,
                               void* ws, size_t ws_bytes, hipStream_t s) {
  AxisPlan p;
  if (!plan_axis(nx, &p) || !plan_axis(ny, &p) || !plan_axis(nz, &p))
    return fail(RISM3D_E_ARG, "grid %dx%dx%d unsupported", nx, ny, nz);
  if (count < 1 || !d_data) return fail(RISM3D_E_ARG, "count < 1 or null data");
  const size_t need = rism3d_transform_workspace_bytes(nx, ny, nz);
  if (!ws || (((uintptr_t)ws) & 255) || ws_bytes < need)
    return fail(RISM3D_E_WORKSPACE, "transform workspace must hold %zu aligned bytes", need);
  return transform_on(nx, ny, nz, count, d_data, forward, ws, s);
}

rism3d_status rism3d_transform_noalloc(int nx, int ny, int nz, int count, void* d_data,
                                       int forward, hipStream_t s) {
  AxisPlan p;
  if (!plan_axis(nx, &p) || !plan_axis(ny, &p) || !plan_axis(nz, &p))
    return fail(RISM3D_E_ARG, "grid %dx%dx%d unsupported", nx, ny, nz);
  if (count < 1 || !d_data) return fail(RISM3D_E_ARG, "count < 1 or null data");
  const size_t need = rism3d_transform_workspace_bytes(nx, ny, nz);
  if (need > kNoAllocScratchBytes)
    return fail(RISM3D_E_ARG, "twiddle tables of %zu bytes exceed the static scratch of %zu",
                need, kNoAllocScratchBytes);
  void* ws = nullptr;
  const rism3d_status st = scratch_address(&ws);
  if (st != RISM3D_OK) return st;
  return transform_on(nx, ny, nz, count, d_data, forward, ws, s);
}

void rism3d_timing_enable(int on) { g_timer.on = on != 0; }

rism3d_status rism3d_timing_select(const char* family) {
  if (!family || !family[0]) {
    g_timer.only = -1;
    return RISM3D_OK;
  }
  for (int f = 0; f < F_COUNT; ++f)
    if (std::strcmp(family, kFamilyNames[f]) == 0) {
      g_timer.only = f;
      return RISM3D_OK;
    }
  return fail(RISM3D_E_ARG, "unknown kernel family '%s'", family);
}

void rism3d_timing_reset(void) {
  for (int f = 0; f < F_COUNT; ++f) {
    g_timer.ms[f] = 0.0;
    g_timer.count[f] = 0;
  }
}

int rism3d_timing_read(int family, const char** name, long* launches, double* total_ms) {
  g_timer.harvest();
  if (family >= 0 && family < F_COUNT) {
    if (name) *name = kFamilyNames[family];
    if (launches) *launches = g_timer.count[family];
    if (total_ms) *total_ms = g_timer.ms[family];
  }
  return F_COUNT;
}

// ---------------------------------------------------------------------------
// Warm-start network
// ---------------------------------------------------------------------------
size_t rism3d_unet_param_count(const rism3d_unet_config* cfg) {
  NetPlan P;
  if (net_plan(cfg, 1 << (cfg ? cfg->levels - 1 : 0), 1 << (cfg ? cfg->levels - 1 : 0),
               1 << (cfg ? cfg->levels - 1 : 0), &P) != RISM3D_OK)
    return 0;
  return P.n_params;
}

size_t rism3d_unet_workspace_bytes(const rism3d_unet_config* cfg, int nx, int ny, int nz,
                                   int training) {
  NetPlan P;
  if (net_plan(cfg, nx, ny, nz, &P) != RISM3D_OK) return 0;
  return training ? P.total_train : P.total_infer;
}

rism3d_status rism3d_unet_forward(const rism3d_unet_config* cfg, int nx, int ny, int nz,
                                  const float* d_params, const float* d_input, float* d_output,
                                  void* d_ws, size_t ws_bytes, hipStream_t s) {
  NetPlan P;
  rism3d_status st = net_plan(cfg, nx, ny, nz, &P);
  if (st != RISM3D_OK) return st;
  if (!d_params || !d_input || !d_output) return fail(RISM3D_E_ARG, "null network buffer");
  if (!d_ws || ((uintptr_t)d_ws & 255)) return fail(RISM3D_E_WORKSPACE, "workspace must be 256-byte aligned");
  if (ws_bytes < P.total_infer)
    return fail(RISM3D_E_WORKSPACE, "network workspace holds %zu bytes, %zu needed", ws_bytes,
                P.total_infer);
  {
    TIMED(F_NET_FWD, s);
    net_pack(P, d_params, d_ws, false, s);
    net_forward(P, d_params, d_input, d_output, d_ws, s);
  }
  LAUNCH_CHECK();
  return RISM3D_OK;
}

rism3d_status rism3d_unet_gradient(const rism3d_unet_config* cfg, int nx, int ny, int nz,
                                   const float* d_params, const float* d_input,
                                   const float* d_target, float* d_grad, double* d_loss,
                                   void* d_ws, size_t ws_bytes, hipStream_t s) {
  NetPlan P;
  rism3d_status st = net_plan(cfg, nx, ny, nz, &P);
  if (st != RISM3D_OK) return st;
  if (!d_params || !d_input || !d_target || !d_grad) return fail(RISM3D_E_ARG, "null network buffer");
  if (!d_ws || ((uintptr_t)d_ws & 255)) return fail(RISM3D_E_WORKSPACE, "workspace must be 256-byte aligned");
  if (ws_bytes < P.total_train)
    return fail(RISM3D_E_WORKSPACE, "network workspace holds %zu bytes, %zu needed", ws_bytes,
                P.total_train);
  {
    TIMED(F_NET_GRAD, s);
    net_pack(P, d_params, d_ws, true, s);
    net_gradient(P, d_params, d_input, d_target, d_grad, d_ws, s);
  }
  if (d_loss)
    HIP_TRY(hipMemcpyAsync(d_loss, wsp<double>(d_ws, P.loss), sizeof(double),
                           hipMemcpyDeviceToDevice, s));
  LAUNCH_CHECK();
  return RISM3D_OK;
}

size_t rism3d_unet_adam_scratch_bytes(void) {
  return (size_t)(net::kNormBlocks + 2) * sizeof(double);
}

rism3d_status rism3d_unet_adam(size_t n, float* d_params, float* d_m, float* d_v,
                               const float* d_grad, int step, float lr, float beta1, float beta2,
                               float eps, float clip_norm, double* d_scratch, hipStream_t s) {
  if (!d_params || !d_m || !d_v || !d_grad || n == 0) return fail(RISM3D_E_ARG, "null Adam buffer");
  if (step < 1 || !(lr > 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) ||
      !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f) || !(clip_norm >= 0.0f))
    return fail(RISM3D_E_ARG, "invalid Adam hyper-parameters");
  if (clip_norm > 0.0f && !d_scratch) return fail(RISM3D_E_ARG, "clipping needs the scratch buffer");
  const float c1 = (float)(1.0 - pow((double)beta1, step));
  const float c2 = (float)(1.0 - pow((double)beta2, step));
  const double* scale = nullptr;
  if (clip_norm > 0.0f) {
    hipLaunchKernelGGL(net::k_sumsq, dim3(net::kNormBlocks), dim3(256), 0, s, d_grad, n, d_scratch);
    hipLaunchKernelGGL(net::k_clip_scale, dim3(1), dim3(64), 0, s, d_scratch, net::kNormBlocks,
                       (double)clip_norm);
    scale = d_scratch + net::kNormBlocks + 1;
  }
  hipLaunchKernelGGL(net::k_adam, dim3(net_blocks(n, 256)), dim3(256), 0, s, d_params, d_m, d_v,
                     d_grad, n, lr, beta1, beta2, eps, c1, c2, scale);
  LAUNCH_CHECK();
  return RISM3D_OK;
}

rism3d_status rism3d_net_input(const rism3d_problem* pr, const rism3d_opts* op, const void* ws_c,
                               size_t ws_bytes, float* d_x, hipStream_t s) {
  Layout L;
  rism3d_status st = make_layout(pr, op, &L);
  if (st != RISM3D_OK) return st;
  if ((st = check_ws(L, ws_c, ws_bytes)) != RISM3D_OK) return st;
  if (!d_x) return fail(RISM3D_E_ARG, "null output");
  const SiteConsts sc = site_consts(pr, L.beta);
  hipLaunchKernelGGL(k_net_input, dim3(blocks_for((size_t)L.nv * L.N, kElemThreads)),
                     dim3(kElemThreads), 0, s, at<float>(ws_c, L.off_w), at<float>(ws_c, L.off_phi),
                     L.N, L.nv, sc, d_x);
  LAUNCH_CHECK();
  return RISM3D_OK;
}

rism3d_status rism3d_csr(const rism3d_problem* pr, const rism3d_opts* op, const void* ws_c,
                         size_t ws_bytes, float* d_c, hipStream_t s) {
  Layout L;
  rism3d_status st = make_layout(pr, op, &L);
  if (st != RISM3D_OK) return st;
  if ((st = check_ws(L, ws_c, ws_bytes)) != RISM3D_OK) return st;
  if (!d_c) return fail(RISM3D_E_ARG, "null output");
  hipLaunchKernelGGL(k_csr_out, dim3(blocks_for((size_t)L.nv * L.N, kElemThreads)),
                     dim3(kElemThreads), 0, s, at<IterState>(ws_c, L.off_state),
                     at<float>(ws_c, L.off_tau), at<float>(ws_c, L.off_tref),
                     at<float>(ws_c, L.off_tlo), at<float>(ws_c, L.off_w), L.N, L.nv,
                     (int)op->closure, order_of(op), d_c);
  LAUNCH_CHECK();
  return RISM3D_OK;
}

rism3d_status rism3d_oz_half_step(const rism3d_problem* pr, const rism3d_opts* op,
                                  const float* d_c0, float c_scale, void* ws, size_t ws_bytes,
                                  float* d_tau0, hipStream_t s) {
  Layout L;
  rism3d_status st = make_layout(pr, op, &L);
  if (st != RISM3D_OK) return st;
  if ((st = check_ws(L, ws, ws_bytes)) != RISM3D_OK) return st;
  if (!d_c0 || !d_tau0) return fail(RISM3D_E_ARG, "null buffer");
  TIMED(F_HALFSTEP, s);
  hipLaunchKernelGGL(k_pack_c64, dim3(blocks_for((size_t)L.npair * L.N, kElemThreads)),
                     dim3(kElemThreads), 0, s, d_c0, L.N, L.nv, (double)c_scale,
                     at<double2>(ws, L.off_spec));
  launch_fft3<double2>(L, ws, 1, nullptr, s);
  launch_contract(L, ws, true, (1.0 / pr->dk), nullptr, s);
  launch_fft3<double2>(L, ws, 0, nullptr, s);
  hipLaunchKernelGGL(k_tau_from_h, dim3(blocks_for((size_t)L.nv * L.N, kElemThreads)),
                     dim3(kElemThreads), 0, s, at<double2>(ws, L.off_spec), d_c0, L.N, L.nv,
                     (double)c_scale, d_tau0);
  LAUNCH_CHECK();
  return RISM3D_OK;
}

rism3d_status rism3d_warmstart(const rism3d_problem* pr, const rism3d_opts* op,
                               const rism3d_unet_config* cfg, const float* d_params, float c_scale,
                               void* ws, size_t ws_bytes, void* d_net_ws, size_t net_ws_bytes,
                               float* d_tau0, hipStream_t s) {
  Layout L;
  rism3d_status st = make_layout(pr, op, &L);
  if (st != RISM3D_OK) return st;
  if ((st = check_ws(L, ws, ws_bytes)) != RISM3D_OK) return st;
  if (!cfg || cfg->in_channels != L.nv || cfg->out_channels != L.nv)
    return fail(RISM3D_E_ARG, "network channels must equal the number of solvent sites");
  // the network input and its prediction use two per-site grids of the
  // workspace that the next solve overwrites (reference tau and residual)
  float* x = at<float>(ws, L.off_tref);
  float* c0 = at<float>(ws, L.off_rref);
  if ((st = rism3d_net_input(pr, op, ws, ws_bytes, x, s)) != RISM3D_OK) return st;
  if ((st = rism3d_unet_forward(cfg, L.nx, L.ny, L.nz, d_params, x, c0, d_net_ws, net_ws_bytes,
                                s)) != RISM3D_OK)
    return st;
  return rism3d_oz_half_step(pr, op, c0, c_scale, ws, ws_bytes, d_tau0, s);
}

rism3d_status rism3d_autotune(const rism3d_problem* pr, const rism3d_opts* op, void* ws,
                              size_t ws_bytes, rism3d_tuning* out, hipStream_t s) {
  Layout L;
  rism3d_status st = make_layout(pr, op, &L);
  if (st != RISM3D_OK) return st;
  if ((st = check_ws(L, ws, ws_bytes)) != RISM3D_OK) return st;
  rism3d_tuning res;
  memset(&res, 0, sizeof(res));
  if (!(fixed_fft_size(L.nx) && fixed_fft_size(L.ny) && zcz_supported(L))) {
    if (out) *out = res;
    return RISM3D_OK;   // no tunable kernels on this grid
  }
  const bool timing = g_timer.on;
  g_timer.on = false;
  float2* spec = at<float2>(ws, L.off_spec);
  const float2* tw = at<float2>(ws, L.off_tw32[1]);
  HIP_TRY(hipMemsetAsync(spec, 0, (size_t)L.npair * L.N * sizeof(float2), s));
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  const double inv_dkt = (1.0 / pr->dk);
  constexpr int kReps = 10;
  auto time_us = [&](auto&& launch) -> double {
    for (int r = 0; r < 2; ++r) launch();
    (void)hipEventRecord(e0, s);
    for (int r = 0; r < kReps; ++r) launch();
    (void)hipEventRecord(e1, s);
    (void)hipEventSynchronize(e1);
    float ms = 0.0f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    return 1e3 * ms / kReps;
  };
  const int y_cands[] = {0, 8, 16, 32, 64};
  const int z_cands[] = {0, 4, 8, 16};
  const int x_cands[] = {0, 8, 16, 32};
  double best_y = 1e30, best_z = 1e30, best_x = 1e30;
  // fused x kernels: zeroed history and reference grids and a steady-state
  // MDIIS state (the potential stays; the workspace's solution is not kept,
  // the next rism3d_solve starts afresh)
  HIP_TRY(hipMemsetAsync(at<char>(ws, L.off_tau), 0, L.off_spec - L.off_tau, s));
  hipLaunchKernelGGL(k_tune_state, dim3(1), dim3(1), 0, s, at<IterState>(ws, L.off_state), L.M,
                     (float)op->mdiis_eta);
  for (int c : x_cands) {
    const double us = time_us([&] {
      launch_fused<false>(L, ws, op, true, s, Batch{}, c, false);
      launch_fused<false>(L, ws, op, false, s, Batch{}, c, false);
    });
    if (c == 0) res.x_default_us = us;
    if (us < best_x) { best_x = us; res.x_lines = c; }
  }
  for (int c : y_cands) {
    if (c == 64 && L.ny > 128) continue;
    const double us = time_us([&] { launch_y32(L, spec, tw, 1, nullptr, s, Batch{}, c); });
    if (c == 0) res.y_default_us = us;
    if (us < best_y) { best_y = us; res.y_lines = c; }
  }
  for (int c : z_cands) {
    const double us =
        time_us([&] { launch_zcz<float2>(L, ws, inv_dkt, nullptr, s, Batch{}, c); });
    if (c == 0) res.z_default_us = us;
    if (us < best_z) { best_z = us; res.z_cols = c; }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  g_timer.on = timing;
  LAUNCH_CHECK();
  res.y_us = best_y;
  res.z_us = best_z;
  res.x_us = best_x;
  set_tune(L, Tune{res.y_lines, res.z_cols, res.x_lines});
  rism3d_release_graphs();   // captured graphs hold the previous kernels
  if (out) *out = res;
  return RISM3D_OK;
}

rism3d_status rism3d_tune_set(const rism3d_problem* pr, const rism3d_opts* op, int y_lines,
                              int z_cols, int x_lines) {
  Layout L;
  rism3d_status st = make_layout(pr, op, &L);
  if (st != RISM3D_OK) return st;
  if (!(y_lines == 0 || y_lines == 8 || y_lines == 16 || y_lines == 32 || y_lines == 64) ||
      !(z_cols == 0 || z_cols == 4 || z_cols == 8 || z_cols == 16) ||
      !(x_lines == 0 || x_lines == 8 || x_lines == 16 || x_lines == 32))
    return fail(RISM3D_E_ARG,
                "y_lines must be 0, 8, 16, 32 or 64, z_cols 0, 4, 8 or 16, x_lines 0, 8, 16 or 32");
  set_tune(L, Tune{y_lines, z_cols, x_lines});
  rism3d_release_graphs();
  return RISM3D_OK;
}

void rism3d_tune_reset(void) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  g_tunes.clear();
  rism3d_release_graphs();
}

const char* rism3d_last_error(void) { return g_error.c_str(); }

void rism3d_constants(double* coulomb, double* kboltz, double* screen, double* d_min,
                      double* beta_u_cap) {
  if (coulomb) *coulomb = kCoulomb;
  if (kboltz) *kboltz = kBoltzmann;
  if (screen) *screen = kScreen;
  if (d_min) *d_min = kDMin;
  if (beta_u_cap) *beta_u_cap = kBetaUCap;
}

}  // extern "C"
