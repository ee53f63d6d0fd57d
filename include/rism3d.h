/*
 * rism3d.h -- C ABI of the MI355X (gfx950) 3D-RISM solver library.
 *
 * The library solves the 3D-RISM equations of arXiv 2403.01039 for one solute
 * in a multi-site solvent on a uniform 3D grid:
 *   - Eq 13  h_g(r) = sum_g' c_g' * chi_g'g            (3D-RISM equation)
 *   - Eq 14-16 closures (HNC, KH) plus PSE-n (Kast & Kloss 2008)
 *   - Eq 22  solute-solvent LJ + Coulomb potential
 *   - Eq 29-30 analytic long-range split, half-integer k grid
 *   - Eq 31-33 and steps 1-7 of "Numerical procedure"
 *   - Eq 40  MDIIS acceleration, Eq 41 RMS stopping rule
 *   - Eq 17-18 solvation free energy.
 *
 * Units: Angstrom, kcal/mol, elementary charge, Kelvin.
 *
 * Memory model.  Every large buffer is caller-owned device memory (for example
 * a torch tensor): the solute atoms, the solvent susceptibility table, the
 * workspace and the output grids.  Per-site solvent parameters (at most
 * RISM3D_MAX_SITES) are small host arrays read during the call.  The library
 * allocates no device memory.  Calls are ordered on the given HIP stream;
 * rism3d_solve and rism3d_thermo synchronise that stream to return their
 * small host-side results (iteration info, free energies).
 *
 * Errors.  Every entry point returns a rism3d_status; nothing throws across the
 * ABI.  rism3d_last_error() returns a thread-local message for the last
 * failing call on the calling thread.
 *
 * Grid layout.  All grids are site-major, x fastest: index
 *   ((site * nz + iz) * ny + iy) * nx + ix.
 * Grid point (ix, iy, iz) sits at r = center + ((ix - nx/2), (iy - ny/2),
 * (iz - nz/2)) * spacing (integer division), so the box centre is a grid
 * point and the box spans [center - (n/2) spacing, center + (n - n/2) spacing).
 */
#ifndef RISM3D_H
#define RISM3D_H

#include <stddef.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RISM3D_MAX_SITES 8
#define RISM3D_MAX_DEPTH 16
#define RISM3D_HISTORY_LEN 16384  /* residual history entries kept per workspace */

typedef enum {
  RISM3D_OK = 0,
  RISM3D_E_ARG = 1,          /* invalid argument (sizes, pointers, options) */
  RISM3D_E_DEVICE = 2,       /* a HIP call failed */
  RISM3D_E_NOCONV = 3,       /* max_iter reached; info and outputs hold the last iterate */
  RISM3D_E_NONFINITE = 4,    /* the residual became NaN/Inf */
  RISM3D_E_WORKSPACE = 5     /* workspace too small or not prepared by rism3d_potential */
} rism3d_status;

typedef enum { RISM3D_KH = 0, RISM3D_HNC = 1, RISM3D_PSE = 2 } rism3d_closure;

/* The problem statement (Eq 22 for the solute, Eq 13 for the solvent).
 *
 * Solute atoms (device pointers, float64): xyz[n_atoms][3] (A), q (e),
 * sigma (A), eps (kcal/mol).  Lorentz-Berthelot mixing with the solvent sites.
 *
 * Solvent sites (host pointers, float64, n_sites <= RISM3D_MAX_SITES):
 * site_q (e), site_sigma (A), site_eps (kcal/mol), site_rho (number density of
 * the species the site belongs to, A^-3).
 *
 * chi (device pointer, float64): chi[(a * n_sites + b) * n_k + m] =
 * chi_ab(m * dk), the solvent susceptibility w_ab + rho_a h_ab from a 1D RISM
 * solvent calculation, on a uniform k grid (dk in A^-1).  The table must reach
 * past the largest |k| of the grid: (n_k - 1) * dk >= |k|_max.
 *
 * Grid: nx, ny, nz points (each even, 2..512, with prime factors 2, 3 and 5
 * only; an odd axis would have a self-mirrored half-integer frequency at which
 * the analytic long-range spectrum of Eq 30 is not Hermitian), spacing in A,
 * center in A.
 */
typedef struct {
  int n_atoms;
  const double* xyz;
  const double* q;
  const double* sigma;
  const double* eps;
  int n_sites;
  const double* site_q;
  const double* site_sigma;
  const double* site_eps;
  const double* site_rho;
  int n_k;
  double dk;
  const double* chi;
  double temperature;
  int nx, ny, nz;
  double spacing;
  double center[3];
  double compressibility;  /* chi_T of the bulk solvent (Eq 19), A^3 mol/kcal; 0: unknown */
  double pressure;         /* bulk solvent pressure (Eq 20), kcal/(mol A^3) */
} rism3d_problem;

/* Solver options (Eq 40-41 and the closure choice).
 * closure, pse_order (PSE-n order n >= 1; PSE-1 is KH), tol (RMS residual
 * threshold, Eq 41; the paper's default is 1e-6), max_iter, mdiis_depth
 * (1..RISM3D_MAX_DEPTH), mdiis_eta (damping of the MDIIS step, (0, 2]),
 * eta_dynamic (non-zero: eta = clamp(-0.2 ln RMS, 0.1, 1.0) each step),
 * check_every (host polls the device convergence flag every this many
 * iterations; 0 picks a default), anchor_every (every this many iterations the
 * residual is evaluated exactly in FP64 and the FP32 iterations in between
 * transform only the increment from that anchor; 0 picks the default, 32),
 * accelerator (RISM3D_MDIIS, or RISM3D_ANDERSON: the modified Anderson method
 * with two histories of section "Convergence acceleration", Eq 34-39: Picard
 * for the first two steps, then theta from Eq 36 in the inner product of
 * Eq 38 with weights 1/rho_g, shifts anderson_s1 and anderson_s2 (the paper
 * uses 0.2 and 0.0) and mixing b = mdiis_eta (the paper uses 0.6); it keeps
 * three (tau, R) pairs whatever mdiis_depth says). */
typedef enum { RISM3D_MDIIS = 0, RISM3D_ANDERSON = 1 } rism3d_accelerator;
typedef struct {
  rism3d_closure closure;
  int pse_order;
  double tol;
  int max_iter;
  int mdiis_depth;
  double mdiis_eta;
  int eta_dynamic;
  int check_every;
  int anchor_every;
  rism3d_accelerator accelerator;
  double anderson_s1, anderson_s2;
} rism3d_opts;

typedef struct {
  int iterations;       /* evaluations of the 3D-RISM map (steps 2-5) */
  double rms;           /* RMS residual of the returned iterate; on convergence always that
                           of an exact FP64 evaluation of the map at it (see rism3d_solve) */
  int restarts;         /* MDIIS restarts */
  int warm_start_used;  /* 1 if a caller tau0 was used */
} rism3d_info;

typedef struct {
  double sfe;                         /* kcal/mol, Eq 17 / Eq 18 / PSE-n */
  double sfe_site[RISM3D_MAX_SITES];  /* per-site contributions */
  double rho_int_c[RISM3D_MAX_SITES]; /* rho_g \int c_g(r) dr (box sum, full c), per site */
  double rho_int_c_total;             /* their sum */
  double pmv;     /* Eq 19: k_B T chi_T (1 - rho_int_c_total), A^3; NaN if compressibility is 0 */
  double pc;      /* Eq 21: -pressure * pmv, kcal/mol (NaN likewise) */
  double sfe_pc;  /* sfe + pc */
} rism3d_thermo_out;

/* Bytes of device workspace needed for this problem and options. Returns 0 on
 * invalid arguments (see rism3d_last_error). */
size_t rism3d_workspace_bytes(const rism3d_problem* problem, const rism3d_opts* opts);

/* Eq 22 and Eq 29-30: fills the workspace with, per solvent site g,
 *   w_g(r) = min(beta u_g(r), 1e4) - f_g(r)   (float32 [n_sites][nz][ny][nx]),
 *   phi_lr(r) = sum_a q_a (1 - exp(-|r - R_a|)) / |r - R_a|   (f_g = beta C q_g phi_lr),
 * the analytic long-range spectrum of Eq 30 on the half-integer k grid, the
 * interpolation tables of chi and the FFT twiddles.  d_ws must be 256-byte
 * aligned and hold rism3d_workspace_bytes(problem, opts) bytes (the options
 * fix the MDIIS history size).  Must precede rism3d_solve on the same
 * workspace. */
rism3d_status rism3d_potential(const rism3d_problem* problem, const rism3d_opts* opts,
                               void* d_ws, size_t ws_bytes, hipStream_t stream);

/* Steps 1-7 of "Numerical procedure" with MDIIS (Eq 40) or, when
 * opts->accelerator is RISM3D_ANDERSON, the modified Anderson method
 * (Eq 34-39).  d_tau0 (device, float32
 * [n_sites][nz][ny][nx], may be NULL) is the starting short-range indirect
 * correlation tau = t - f; NULL starts from t = f (tau = 0) as the paper does.
 * On return d_g (device, float32 [n_sites][nz][ny][nx], may be NULL) holds
 * g_g(r) of the returned iterate, and info (host, may be NULL) the iteration
 * count, final RMS and restart count.  Returns RISM3D_E_NOCONV when max_iter
 * is reached (outputs then hold the last iterate), RISM3D_E_NONFINITE on a
 * NaN/Inf residual.
 * Stopping rule (Eq 41).  The bulk iterations evaluate the map in FP32 as an
 * increment over the last FP64 evaluation (every anchor_every iterations),
 * so their residual is an estimate.  When an estimate falls below tol, the
 * next evaluation is an exact FP64 one of that same iterate, and only an FP64
 * residual below tol ends the solve: the returned iterate's exact residual
 * (the info->rms reported) is below tol.  That evaluation counts as an
 * iteration and may run one past max_iter. */
rism3d_status rism3d_solve(const rism3d_problem* problem, const rism3d_opts* opts,
                           const float* d_tau0, void* d_ws, size_t ws_bytes, float* d_g,
                           rism3d_info* info, hipStream_t stream);

/* A closure ladder (continuation in the closure): rism3d_solve under
 * stages[0], then under stages[1], ... on one workspace.  Stage 0 starts
 * from d_tau0 (or t = f when NULL); every later stage starts from the
 * iterate the stage before returned (tau rounded to float32).  The usual
 * ladder is KH, then PSE-2, then PSE-n with each stage's own tolerance and
 * damping: a high-order PSE closure (Kast & Kloss) or HNC (Eq 14) started
 * from t = f can diverge where KH (Eq 15) converges.  Every stage must give
 * the workspace layout of stages[0] (same MDIIS depth and accelerator);
 * closure, order, tol, max_iter and damping may differ; a stage may repeat
 * the one before (the next stage starts with an empty MDIIS history).  info
 * (host, may be NULL) receives n_stages entries.  A stage that reaches its
 * max_iter (RISM3D_E_NOCONV) still hands its last iterate to the next stage;
 * any other failing status ends the ladder with it (later entries of info
 * are not written).  The ladder's status is the last stage's.  d_g (may be
 * NULL) receives g of the last stage, and rism3d_thermo with the last
 * stage's options evaluates its free energy. */
rism3d_status rism3d_solve_ladder(const rism3d_problem* problem, const rism3d_opts* stages,
                                  int n_stages, const float* d_tau0, void* d_ws, size_t ws_bytes,
                                  float* d_g, rism3d_info* info, hipStream_t stream);

/* Many solutes in one call: for each of the n problems (host array; any mix
 * of solutes, grids and solvents, one set of options), the work of
 * rism3d_potential, rism3d_solve and (if thermo != NULL) rism3d_thermo.
 * Problems whose iteration layout agrees (grid, sites, MDIIS depth,
 * susceptibility table length and spacing) and whose axis lengths are in
 * {32, 64, 96, 128, 192, 256, 512} with nz in {64, 96, 128, 256} form a
 * group; each kernel of an iteration is launched once per group, with one
 * slab of workgroups per member, and a converged member's workgroups exit at
 * once while the others iterate.  Other problems iterate as groups of one.
 * The host reads the members' states after each anchor period.
 *   d_ws: one device workspace of rism3d_batch_workspace_bytes(n, ...) bytes,
 *         256-byte aligned, owned by the caller (0 is returned for invalid
 *         problems or options, with the reason in rism3d_last_error).
 *   d_tau0: NULL, or a host array of n device pointers (entries may be NULL)
 *         to starting tau fields as for rism3d_solve.
 *   d_g: NULL, or a host array of n device pointers (entries may be NULL)
 *         receiving g of each member.
 *   info, thermo: NULL, or host arrays of n results.
 * Returns RISM3D_OK when every member converged; otherwise the status of the
 * first non-converged member (RISM3D_E_NONFINITE before RISM3D_E_NOCONV),
 * with every member's results still written. */
size_t rism3d_batch_workspace_bytes(int n, const rism3d_problem* problems,
                                    const rism3d_opts* opts);
rism3d_status rism3d_solve_batch(int n, const rism3d_problem* problems, const rism3d_opts* opts,
                                 const float* const* d_tau0, void* d_ws, size_t ws_bytes,
                                 float* const* d_g, rism3d_info* info, rism3d_thermo_out* thermo,
                                 hipStream_t stream);

/* Eq 17 (HNC), Eq 18 (KH) and the PSE-n form: the solvation free energy of the
 * iterate rism3d_solve returned, as k_B T sum_g rho_g dV sum_r Phi_g(r) with
 * h = g - 1 and c = g - 1 - t, accumulated in float64; in the same pass the
 * integrals rho_g dV sum_r c_g(r) of Eq 19.  From them and the problem's bulk
 * compressibility and pressure: the partial molar volume (Eq 19) and the PC
 * term -P V (Eq 21).  Writes out (host). */
rism3d_status rism3d_thermo(const rism3d_problem* problem, const rism3d_opts* opts,
                            const void* d_ws, size_t ws_bytes, rism3d_thermo_out* out,
                            hipStream_t stream);

/* Section "Hybrid implementation", the derivative of the MM/3D-RISM free
 * energy (Eq 23): the solvent term
 *   d(dmu)/dR_a = sum_g rho_g \int g_g(r) du_g(r)/dR_a dr
 * for every solute atom a, with u_g the potential of Eq 22 (distances clamped
 * at 0.01 A, so pairs closer than that add nothing) and the integral taken as
 * the box sum dV sum_r.  The solvation force on atom a is minus this.
 *   d_g:    device, float32 [n_sites][nz][ny][nx], any distribution (normally
 *           the g that rism3d_solve wrote); read only.
 *   d_grad: device, float64 [n_atoms][3] (x, y, z), kcal/(mol A); written.
 *           May be NULL when n_atoms is 0.
 * The workspace must have been prepared by rism3d_potential (it holds the
 * atoms and their LJ coefficients); the call overwrites the workspace's
 * Fourier scratch, which no later call reads.  Pair terms and sums are
 * float64 and the cross-workgroup sum has a fixed order, so the result is
 * deterministic.  Synchronises the stream (to check the workspace). */
rism3d_status rism3d_sfe_gradient(const rism3d_problem* problem, const rism3d_opts* opts,
                                  const float* d_g, void* d_ws, size_t ws_bytes, double* d_grad,
                                  hipStream_t stream);

/* Copies tau = t - f of the returned iterate (float32 [n_sites][nz][ny][nx]) into
 * d_tau (device); usable as d_tau0 of a later solve (resume / warm start).
 * The solver holds the iterate as a float32 reference plus a float32
 * increment; the copy is their sum rounded to float32, so a solve restarted
 * from it reproduces g to float32 rounding of tau, not bit for bit. */
rism3d_status rism3d_get_tau(const rism3d_problem* problem, const rism3d_opts* opts,
                             const void* d_ws, size_t ws_bytes, float* d_tau,
                             hipStream_t stream);

/* Residual history of the last rism3d_solve on this workspace (Eq 41 per
 * evaluation of the map): rms[i] is the RMS residual of evaluation i + 1 and
 * exact[i] is 1 where that evaluation was an exact FP64 one (an anchor, or
 * the verification of an estimate below tol) and 0 for an FP32 increment
 * estimate.  *count receives the number of evaluations recorded, the
 * iteration count capped at RISM3D_HISTORY_LEN; min(*count, capacity)
 * entries are written to the host arrays rms and exact (which may be NULL
 * when capacity is 0).  Synchronises the stream.  Solves of a batch
 * (rism3d_solve_batch) keep no history readable here. */
rism3d_status rism3d_get_history(const rism3d_problem* problem, const rism3d_opts* opts,
                                 const void* d_ws, size_t ws_bytes, int capacity, double* rms,
                                 int* exact, int* count, hipStream_t stream);

/* One exact (FP64) evaluation of the discretised 3D-RISM map (steps 2-5,
 * Eq 31-33) at tau = t - f: writes the residual R = t' - t = h + 1 - g
 * (device, float32 [n_sites][nz][ny][nx]) and returns its RMS in *rms (host,
 * may be NULL).  d_tau (device, float32, same layout) gives tau; the workspace
 * must be prepared by rism3d_potential and any solution held there is
 * overwritten.  d_tau = NULL evaluates the iterate the last rism3d_solve on
 * this workspace returned, as it is held (FP32 reference + remainder +
 * increment, summed in FP64; rism3d_get_tau would round it to FP32); that
 * solution stays in place. */
rism3d_status rism3d_map(const rism3d_problem* problem, const rism3d_opts* opts, const float* d_tau,
                         void* d_ws, size_t ws_bytes, float* d_residual, double* rms,
                         hipStream_t stream);

/* The map through the kernels of the bulk FP32 iterations, at
 * tau = d_tau_ref + d_delta (both device, float32 [n_sites][nz][ny][nx]): an
 * exact FP64 evaluation at d_tau_ref (the anchor, R_ref), then the FP32
 * evaluation of the increment, R = R_ref + dh - dg with
 * dc = [g(d_ref + delta) - g(d_ref)] - delta transformed in FP32 (Eq 31-33
 * applied to the difference; the long-range term of Eq 32 cancels).  Writes R
 * (device, float32, same layout) and its RMS (host, may be NULL).  Same
 * workspace rules as rism3d_map.  The kernels and tile widths are those a
 * solve of this problem runs, so the FP32 result differs from the exact map
 * at d_tau_ref + d_delta by FP32 round-off of the increment's terms. */
rism3d_status rism3d_map_increment(const rism3d_problem* problem, const rism3d_opts* opts,
                                   const float* d_tau_ref, const float* d_delta, void* d_ws,
                                   size_t ws_bytes, float* d_residual, double* rms,
                                   hipStream_t stream);

/* Copies the fields rism3d_potential computed: w (float32 [n_sites][nz][ny][nx],
 * may be NULL) and phi_lr (float32 [nz][ny][nx], may be NULL), device to device. */
rism3d_status rism3d_get_potential(const rism3d_problem* problem, const rism3d_opts* opts,
                                   const void* d_ws, size_t ws_bytes, float* d_w, float* d_phi,
                                   hipStream_t stream);

/* The half-integer-shifted 3D transform of section "Numerical procedure" on
 * `count` complex grids d_data[count][nz][ny][nx] (device, float2 pairs, in
 * place):  forward != 0:  X_j = sum_a x_a exp(-2 pi i (j + 1/2) . a / n);
 * otherwise the unnormalised inverse  x_a = sum_j X_j exp(+2 pi i (j + 1/2) . a / n).
 * d_ws: device scratch of at least rism3d_transform_workspace_bytes bytes
 * (twiddle tables), 256-byte aligned. */
size_t rism3d_transform_workspace_bytes(int nx, int ny, int nz);
rism3d_status rism3d_transform(int nx, int ny, int nz, int count, void* d_data, int forward,
                               void* d_ws, size_t ws_bytes, hipStream_t stream);

/* rism3d_transform without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, serving loops,
 * harnesses that forbid hipMalloc): the twiddle tables live in a static
 * device array of the library, RISM3D_NOALLOC_SCRATCH_BYTES bytes per GPU,
 * held until the process ends.  Same transform, kernels and results as
 * rism3d_transform.  Axes of up to 512 points (every grid rism3d_transform
 * accepts fits the array).  Allocates nothing and calls no allocating
 * routine.  Runs on the current device, which must be the stream's device.
 * Every call on one GPU rewrites that GPU's tables before its transform, so
 * calls that overlap on one GPU (concurrent streams or threads) race and
 * must be ordered by the caller.  Returns RISM3D_E_ARG for unsupported grids
 * and RISM3D_E_DEVICE when the array's device address cannot be obtained. */
#define RISM3D_NOALLOC_SCRATCH_BYTES (3 * 2 * 512 * 8)
rism3d_status rism3d_transform_noalloc(int nx, int ny, int nz, int count, void* d_data,
                                       int forward, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Learned warm start (not in the paper, which starts every solve at t = f):
 * a 3D convolutional encoder-decoder maps the solute potential of each
 * solvent site to an initial short-range direct correlation c0; one
 * Ornstein-Zernike half-step (Eq 32, Eq 13 and the inverse transform of
 * "Numerical procedure") turns c0 into the starting tau0 = h0 - c0.  The
 * warm start changes only the starting point: the fixed point and its
 * tolerance are those of the plain solve, and rism3d_solve repeats a solve
 * from tau0 = 0 when the iteration from a caller's tau0 ends non-finite.
 *
 * Network: `levels` levels with base * 2^l channels, 3x3x3 convolutions
 * (zero padding), leaky activations of slope `slope`, 2x2x2 average pooling,
 * nearest upsampling, skip concatenation (upsampled channels first):
 *   encoder l: a_l = act(conv(in_l)), e_l = act(conv(a_l)), in_0 = input,
 *              in_{l+1} = pool(e_l);
 *   decoder l = levels-2 .. 0: da_l = act(conv([up(d_{l+1}), e_l])),
 *              d_l = act(conv(da_l)), d_{levels-1} = e_{levels-1};
 *   output = conv(d_0).
 * Parameters: one FP32 vector, per convolution in the order enc0a, enc0b,
 * ..., dec{levels-2}a, dec{levels-2}b, ..., dec0a, dec0b, out: W[C_out][27][C_in]
 * (tap (dz * 3 + dy) * 3 + dx for offsets (dz-1, dy-1, dx-1)) then b[C_out].
 * The kernels run in BF16 on the matrix cores with FP32 accumulation; the
 * parameters, gradients and Adam moments stay FP32.  Grid axes must be
 * multiples of 2^(levels-1); base a multiple of 16 with base * 2^(levels-1)
 * <= 128.  Fields are FP32 site-major [channel][nz][ny][nx] (device).
 * ------------------------------------------------------------------------ */
typedef struct {
  int levels;        /* 4 */
  int base;          /* 16 */
  int in_channels;   /* solvent sites */
  int out_channels;  /* solvent sites */
  float slope;       /* 0.1 */
} rism3d_unet_config;

/* Number of FP32 parameters (0 for an invalid configuration). */
size_t rism3d_unet_param_count(const rism3d_unet_config* cfg);
/* Device workspace bytes for inference (training = 0) or for
 * rism3d_unet_gradient (training != 0) on an nx x ny x nz grid; 0 if invalid. */
size_t rism3d_unet_workspace_bytes(const rism3d_unet_config* cfg, int nx, int ny, int nz,
                                   int training);
/* d_output[out_channels][N] = network(d_params, d_input[in_channels][N]). */
rism3d_status rism3d_unet_forward(const rism3d_unet_config* cfg, int nx, int ny, int nz,
                                  const float* d_params, const float* d_input, float* d_output,
                                  void* d_ws, size_t ws_bytes, hipStream_t stream);
/* Mean squared error of the network output against d_target[out_channels][N]
 * (mean over channels and voxels) and its gradient: d_grad (device,
 * param_count floats) is overwritten; d_loss (device double, may be NULL)
 * receives the loss. */
rism3d_status rism3d_unet_gradient(const rism3d_unet_config* cfg, int nx, int ny, int nz,
                                   const float* d_params, const float* d_input,
                                   const float* d_target, float* d_grad, double* d_loss,
                                   void* d_ws, size_t ws_bytes, hipStream_t stream);
/* One Adam step (Kingma & Ba, bias-corrected, step >= 1) on n parameters.
 * clip_norm > 0 first scales the gradient by min(1, clip_norm / |g|) (global
 * L2 norm, FP64 fixed-order sum); it then needs d_scratch, a device buffer of
 * rism3d_unet_adam_scratch_bytes() bytes, whose last two doubles receive |g|
 * and the applied scale.  clip_norm = 0: no clipping, d_scratch may be NULL. */
size_t rism3d_unet_adam_scratch_bytes(void);
rism3d_status rism3d_unet_adam(size_t n, float* d_params, float* d_m, float* d_v,
                               const float* d_grad, int step, float lr, float beta1, float beta2,
                               float eps, float clip_norm, double* d_scratch, hipStream_t stream);
/* Network input of a prepared workspace: symlog(beta u_g) = sign log(1 + |beta u_g|)
 * of the capped potential, d_x[n_sites][N]. */
rism3d_status rism3d_net_input(const rism3d_problem* problem, const rism3d_opts* opts,
                               const void* d_ws, size_t ws_bytes, float* d_x, hipStream_t stream);
/* Training target of a solved workspace: c_sr = g - 1 - tau of the returned
 * iterate (Eq 31 in tau-form), d_c[n_sites][N]. */
rism3d_status rism3d_csr(const rism3d_problem* problem, const rism3d_opts* opts,
                         const void* d_ws, size_t ws_bytes, float* d_c, hipStream_t stream);
/* tau0 = h0 - s c0 with h0 from c_scale * d_c0 by one Ornstein-Zernike
 * half-step (FP64 transforms and contraction); needs a prepared workspace
 * (rism3d_potential) and uses its spectrum buffer. */
rism3d_status rism3d_oz_half_step(const rism3d_problem* problem, const rism3d_opts* opts,
                                  const float* d_c0, float c_scale, void* d_ws, size_t ws_bytes,
                                  float* d_tau0, hipStream_t stream);
/* The whole warm start on a prepared workspace: network input, inference
 * (network workspace d_net_ws of rism3d_unet_workspace_bytes(.., 0) bytes),
 * c0 = c_scale * output, half-step; writes d_tau0[n_sites][N] for rism3d_solve. */
rism3d_status rism3d_warmstart(const rism3d_problem* problem, const rism3d_opts* opts,
                               const rism3d_unet_config* cfg, const float* d_params, float c_scale,
                               void* d_ws, size_t ws_bytes, void* d_net_ws, size_t net_ws_bytes,
                               float* d_tau0, hipStream_t stream);

/* Autotuning of the FP32 iteration kernels on grids with the fused path:
 * times, on the prepared workspace d_ws (its spectrum buffer is zeroed and
 * used as scratch), the y-pass transform with 8, 16, 32 or 64 lines per
 * workgroup, the z-transform/contraction kernel with 4, 8 or 16 column
 * pairs per workgroup, and the fused update/x-transform and x-transform/
 * residual kernels with 8, 16 or 32 rows per workgroup (widths whose LDS
 * tile would not fit run the default; the workspace's solution is not kept),
 * and keeps the fastest of each for this (nx, ny, nz, n_sites) in a
 * process-wide table that every later solve of that shape uses (cached
 * graphs are released).  The widths change which workgroup transforms a
 * line, not the operations on it: results agree to round-off (separately
 * compiled variants may fuse multiply-adds differently).  out (host, may be
 * NULL) receives the
 * choices (0 = the compiled default) and their times in microseconds.
 * rism3d_tune_set() records given widths for a problem's shape (0 = default;
 * widths without a compiled kernel for that length run the default), and
 * rism3d_tune_reset() restores the defaults for every shape. */
typedef struct {
  int y_lines, z_cols, x_lines;
  double y_us, z_us, x_us, y_default_us, z_default_us, x_default_us;
} rism3d_tuning;
rism3d_status rism3d_autotune(const rism3d_problem* problem, const rism3d_opts* opts, void* d_ws,
                              size_t ws_bytes, rism3d_tuning* out, hipStream_t stream);
rism3d_status rism3d_tune_set(const rism3d_problem* problem, const rism3d_opts* opts, int y_lines,
                              int z_cols, int x_lines);
void rism3d_tune_reset(void);

/* Kernel timing, for profiling (thread-local switch).  While enabled, calls on
 * this thread record a pair of HIP events on the call's stream around every
 * kernel launch and add the elapsed time to a per-family total when the call
 * synchronises.  rism3d_timing_read(i, ...) fills the name, launch count and
 * total milliseconds of family i and returns the number of families (call with
 * i = -1 to get the count only).  Enabling costs two event records per timed
 * launch (each record also orders the stream, so timing every family slows a
 * solve by about a tenth).  rism3d_timing_select(name) restricts the events to
 * the one family of that name (NULL or "" restores every family); an unknown
 * name returns RISM3D_E_ARG and leaves the selection unchanged. */
void rism3d_timing_enable(int on);
rism3d_status rism3d_timing_select(const char* family);
void rism3d_timing_reset(void);
int rism3d_timing_read(int family, const char** name, long* launches, double* total_ms);

/* Execution of the iteration: by default one anchor period of iterations is
 * captured into a HIP graph the first time a (workspace, problem shape,
 * options) combination is solved and replayed afterwards (the graph is keyed
 * by the workspace address and layout, which fix every kernel argument, and
 * touches no memory outside the workspace).  rism3d_use_graphs(0)
 * launches the kernels directly instead.  rism3d_release_graphs() destroys
 * the library-owned graph cache (host-side handles). */
void rism3d_use_graphs(int on);
void rism3d_release_graphs(void);

/* Thread-local message describing the last error on this thread ("" if none). */
const char* rism3d_last_error(void);

/* The unit constants the library uses: Coulomb factor C (kcal A / (mol e^2)),
 * Boltzmann constant (kcal / (mol K)), the Eq 29-30 screening length (A), the
 * distance clamp (A) and the cap on beta*u.  Host only; no device access. */
void rism3d_constants(double* coulomb, double* kboltz, double* screen, double* d_min,
                      double* beta_u_cap);

#ifdef __cplusplus
}
#endif

#endif /* RISM3D_H */
