// Shared device/host definitions of the gfx950 3D-RISM library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "../../include/rism3d.h"

namespace rism {

// Unit conventions (kcal/mol, Angstrom, e).  Eq 22 is printed without the
// Coulomb factor; C is the CODATA 2018 value in these units.
constexpr double kCoulomb = 332.0637133;     // kcal A / (mol e^2)
constexpr double kBoltzmann = 0.0019872043;  // kcal / (mol K)
constexpr double kScreen = 1.0;              // A, screening length of Eq 29-30
constexpr double kDMin = 0.01;               // A, distance clamp in Eq 22
constexpr double kBetaUCap = 1.0e4;          // cap on beta*u before f is removed
static_assert(kScreen == 1.0, "the potential kernel evaluates (1 - e^{-d/l})/d with l = 1 A");

constexpr int kMaxSites = RISM3D_MAX_SITES;
constexpr int kMaxDepth = RISM3D_MAX_DEPTH;
constexpr int kHistLen = RISM3D_HISTORY_LEN;
constexpr int kMaxRadixPasses = 12;

// Solvent-site constants passed by value to kernels.
struct SiteConsts {
  int nv;
  float coul[kMaxSites];     // beta C q_g  (f_g = coul[g] * phi_lr)
  double coul64[kMaxSites];
  double q64[kMaxSites];
  double rho[kMaxSites];
};

// Per-site weights of the Gram inner product: 1 for MDIIS (unweighted), 1/rho
// for modified Anderson (Eq 38).  The RMS of Eq 41 stays unweighted.
struct GramW {
  float w[kMaxSites];
};

// Solvent-site LJ parameters (Lorentz-Berthelot mixing with each solute atom).
struct SiteLJ {
  double sigma[kMaxSites];
  double eps[kMaxSites];
};

// An FFT axis: length and radix plan (product of radices == n).
struct AxisPlan {
  int n;
  int npass;
  int radix[kMaxRadixPasses];
};

// Device-resident MDIIS / iteration state (one per workspace).
struct IterState {
  double gram[kMaxDepth][kMaxDepth];  // <R_i, R_j>, unnormalised
  double rms_slot[kMaxDepth];
  double last_rms;
  double last_rr;
  float coef[kMaxDepth];              // coefficients of the next update (0 = unused)
  float eta;                          // damping of the next update
  int stored[kMaxDepth];              // slot holds a (tau, R) pair
  int stamp[kMaxDepth];               // insertion order of stored pairs
  int stamp_counter;
  int dest;                           // slot receiving the next tau
  int newest;                         // most recently stored slot (difference-form update)
  int iter;                           // completed map evaluations
  int done;                           // kDoneFinished, kDoneVerify or 0 (iterate)
  int converged;
  int status;                         // rism3d_status of the iteration
  int restarts;
  int final_slot;                     // slot of the accepted iterate
  int warm;                           // 1 if a caller tau0 seeded iteration 0
  int prepared;                       // magic set by rism3d_potential
  unsigned layout_key;                // digest of the workspace layout it was prepared with
  int ticket;                         // workgroups of the fused residual kernel that finished
  int hold;                           // the next update re-evaluates the iterate in slot dest
};

// IterState::done.  kDoneVerify: an FP32 evaluation (whose residual is an
// estimate built from increments) passed the tolerance; the FP32 kernels then
// skip, and the next FP64 anchor evaluation re-evaluates that same iterate
// exactly and decides.  Only an FP64 evaluation finishes a converged solve.
constexpr int kDoneFinished = 1;
constexpr int kDoneVerify = 2;

// Whether a kernel of an FP64 (anchor) or FP32 evaluation skips its work.
template <bool F64>
__device__ __forceinline__ bool skip_iteration(int done) {
  return F64 ? done == kDoneFinished : done != 0;
}

constexpr int kPreparedMagic = 0x52495344;  // "RISD"

// Complex helpers for float2 (bulk FP32 path) and double2 (FP64 anchors).
#define RISM_CPLX_OPS(C, S, MAKE)                                                              \
  __host__ __device__ inline C cmul(C a, C b) { return MAKE(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); } \
  __host__ __device__ inline C cmulc(C a, C b) { return MAKE(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y); } \
  __host__ __device__ inline C cadd(C a, C b) { return MAKE(a.x + b.x, a.y + b.y); }          \
  __host__ __device__ inline C csub(C a, C b) { return MAKE(a.x - b.x, a.y - b.y); }          \
  __host__ __device__ inline C cscale(C a, S s) { return MAKE(a.x * s, a.y * s); }            \
  __host__ __device__ inline C cconj(C a) { return MAKE(a.x, -a.y); }                         \
  /* sgn * i * a */                                                                           \
  __host__ __device__ inline C cmul_i(C a, S sgn) { return MAKE(-sgn * a.y, sgn * a.x); }

RISM_CPLX_OPS(float2, float, make_float2)
RISM_CPLX_OPS(double2, double, make_double2)
#undef RISM_CPLX_OPS

template <typename C> struct ScalarOf;
template <> struct ScalarOf<float2> { using type = float; };
template <> struct ScalarOf<double2> { using type = double; };

__host__ __device__ inline float2 make_c(float x, float y) { return make_float2(x, y); }
__host__ __device__ inline double2 make_c(double x, double y) { return make_double2(x, y); }

// Closures (Eq 14; KH with exp below 0 and linear above; PSE-n series above 0),
// in the precision of the argument.
template <typename S>
__device__ inline S closure_g(S d, int kind, int order) {
  if (kind == RISM3D_HNC) return exp(d);
  if (d <= S(0)) return exp(d);
  if (kind == RISM3D_KH) return S(1) + d;
  S term = S(1), sum = S(1);
  for (int i = 1; i <= order; ++i) {
    term = term * d / (S)i;
    sum += term;
  }
  return sum;
}

// g(d_ref + delta) - g(d_ref) without cancellation: on the exponential branch
// e^{d_ref} expm1(delta); on the linear KH branch delta; on the PSE-n series
// branch the exact Taylor expansion sum_j delta^j / j! * g_{n-j}(d_ref).
// Where the two points straddle 0 the plain difference is used (|d| <= |delta|).
__device__ inline float closure_dg(float dref, float delta, int kind, int order) {
  const float dnew = dref + delta;
  if (kind == RISM3D_HNC || (dref <= 0.0f && dnew <= 0.0f)) {
    // For a large step the plain difference has no cancellation, and it avoids
    // 0 * inf when e^{d_ref} underflows inside the core.
    if (delta > 16.0f) return expf(dnew) - expf(dref);
    return expf(dref) * expm1f(delta);
  }
  if (dref > 0.0f && dnew > 0.0f) {
    if (kind == RISM3D_KH) return delta;
    float dg = 0.0f, pw = 1.0f;
    for (int j = 1; j <= order; ++j) {
      pw = pw * delta / (float)j;           // delta^j / j!
      float term = 1.0f, part = 1.0f;       // g_{order-j}(dref)
      for (int i = 1; i <= order - j; ++i) {
        term = term * dref / (float)i;
        part += term;
      }
      dg += pw * part;
    }
    return dg;
  }
  return closure_g(dnew, kind, order) - closure_g(dref, kind, order);
}

// Batched launches: blockIdx.y selects the member of a batch whose
// workspaces lie bstride bytes apart (bstride = 0 and one member for a single
// solve).  Null pointers stay null.
template <typename T>
__device__ __forceinline__ T* member_ptr(T* p, size_t bstride) {
  return p ? reinterpret_cast<T*>(reinterpret_cast<uintptr_t>(p) + (size_t)blockIdx.y * bstride)
           : p;
}

// Row width of the susceptibility tables: the nv*nv values of one k-sample,
// padded to whole 16-byte vectors.
template <typename S>
__host__ __device__ constexpr int chi_row(int nv) {
  return sizeof(S) == 4 ? ((nv * nv + 3) & ~3) : ((nv * nv + 1) & ~1);
}

// Workgroups are dispatched round-robin over the 8 XCDs of the chip (block b
// runs on XCD b % 8).  xcd_tile maps block b to a tile index such that each
// XCD takes one contiguous run of tiles, in order; neighbouring tiles that
// share 128-byte lines then meet in the same L2.  A bijection on [0, G).
__device__ __forceinline__ int xcd_tile(int b, int G) {
  constexpr int X = 8;
  const int x = b % X, i = b / X;
  const int q = G / X, r = G % X;
  return x < r ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

}  // namespace rism
