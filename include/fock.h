/*
 * libfock: the Fock exchange operator V_X and the adaptively compressed
 * exchange (ACE) operator on one AMD MI355X (gfx950).
 *
 * The operation (Jia, Wang & Lin, arXiv:1905.01348, Sec. 2, Eq. "applyVX",
 * and the Fock-application algorithm of Sec. 3.2): for orbitals psi_j,
 * j = 0..N-1, and targets phi_k,
 *
 *   (V_X phi_k)(r) = -(1/Omega) sum_j psi_j(r) IFFT_u[ K(G) FFT_u( conj(psi_j) phi_k ) ](r)
 *
 * with FFT_u / IFFT_u the unnormalised DFT pair on the cell's real-space grid,
 * Omega the cell volume and K the Coulomb kernel 4 pi/|G|^2 (K(0) = 0) or the
 * screened kernel 4 pi/|G|^2 (1 - exp(-|G|^2/(4 w^2))) (K(0) = pi/w^2), times
 * the mixing fraction alpha (Sec. 2: V_X[P](r,r') = -alpha P(r,r') K(r-r')).
 * Each (j, k) term is one Poisson-like solve; the paper counts N_e^2 of them
 * per application (Sec. 2).
 *
 * ACE (cited in Sec. 1 as an alternative the paper does not use): from
 * W = V_X Psi, M = Psi^H W (Hermitised), -M = L L^H (Cholesky, L lower with a
 * real positive diagonal), xi = W L^{-H}; K_ACE phi = -xi (xi^H phi).  K_ACE
 * equals V_X on span(Psi).  E_X = 1/2 Re tr(Psi^H V_X Psi) = 1/2 tr M.
 *
 * Conventions shared by every call
 * --------------------------------
 * Layout: a block of orbitals is a device array of interleaved complex values
 *   (re, im).  Column c (orbital c) starts at element base + c*ld, ld >= N_r,
 *   and holds the grid vector with r = ix + n[0]*(iy + n[1]*iz), x fastest.
 *   A contiguous torch tensor of shape (N, nz, ny, nx) has ld = N_r.
 * Normalisation: orbitals are Euclidean-orthonormal grid vectors
 *   (sum_r conj(psi_i) psi_j = delta_ij); the prefactor is -1/Omega.  The
 *   library does not check orthonormality.
 * Ownership: psi, phi and out are caller-owned device memory; the library
 *   never frees them and keeps no reference past the stream-ordered end of
 *   the call.  Outputs are overwritten, never accumulated into; out must not
 *   alias psi or phi.  An fx_ace owns its factors until fx_ace_free.
 * Streams: calls enqueue on `stream` (a hipStream_t; NULL means the default
 *   (null) stream, as everywhere in HIP) and return without waiting, except fx_build_ace (one wait, to
 *   read the Cholesky status) and fx_serve (runs to completion).  Workspace
 *   is allocated on the first use of a shape, inside the context's HBM
 *   budget; a later call with a shape already seen allocates nothing.
 * Graph capture: fx_apply_vx and fx_apply_ace may be captured into a HIP
 *   graph once the same call (same grid, kernel, precisions and sizes) has
 *   run outside capture on the same context or fx_ace; a captured call that
 *   would have to allocate or upload tables fails with FX_ERR_INVALID
 *   instead.  The graph holds the workspace addresses of the time of
 *   capture: a later uncaptured call that needs a larger workspace on that
 *   context (or fx_ace) reallocates it, and graphs captured before must not
 *   be replayed after that.  Per-kernel timing skips captured launches.
 *   fx_build_ace and fx_serve wait on the host and refuse capture.
 * Errors: every call returns an fx_status.  Argument errors are reported
 *   synchronously before anything is enqueued; a text description of the
 *   last error on the calling thread is available from fx_last_error().
 *   HIP runtime failures map to FX_ERR_DEVICE.
 * Threads: one fx_ctx per host thread, or external locking.
 */
#ifndef LIBFOCK_FOCK_H
#define LIBFOCK_FOCK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum fx_status {
  FX_OK = 0,
  FX_ERR_INVALID = -1,     /* null pointer, bad size or leading dimension, aliasing */
  FX_ERR_UNSUPPORTED = -2, /* grid edge not of the form 2^a 3^b in [2, 96], unknown enum */
  FX_ERR_OOM = -3,         /* allocation failed or the HBM budget is exhausted */
  FX_ERR_NOT_POSDEF = -4,  /* -M is not Hermitian positive definite (ACE build) */
  FX_ERR_DEVICE = -5,      /* a HIP runtime call failed */
  FX_ERR_BUSY = -6,        /* serving: request refused by admission control */
  FX_ERR_CANCELLED = -7    /* serving: request cancelled before it ran */
} fx_status;

typedef enum fx_dtype {
  FX_C128 = 0, /* complex double, interleaved */
  FX_C64 = 1   /* complex float, interleaved */
} fx_dtype;

typedef enum fx_kernel_kind {
  FX_COULOMB = 0, /* K = 4 pi/|G|^2, K(0) = 0 */
  FX_HSE = 1      /* K = 4 pi/|G|^2 (1 - exp(-|G|^2/(4 w^2))), K(0) = pi/w^2 */
} fx_kernel_kind;

typedef enum fx_prec {
  /* V_X pair path */
  FX_PREC_FP64 = 0,       /* FP64 FFTs, FP64 accumulation */
  FX_PREC_FP32 = 1,       /* FP32 FFTs, FP32 accumulation */
  FX_PREC_FP32_ACC64 = 2, /* FP32 FFTs, FP64 accumulation over j */
  /* ACE GEMMs */
  FX_PREC_ACE_FP64 = 3,   /* FP64 matrix cores */
  FX_PREC_ACE_FP32R = 4,  /* FP32 matrix cores + one FP64-combined residual step */
  FX_PREC_ACE_BF16R = 5,  /* BF16 matrix cores + one FP64-combined residual step */
  FX_PREC_ACE_FP32 = 6,   /* FP32 matrix cores, no residual step (ablation) */
  FX_PREC_ACE_BF16 = 7,   /* BF16 matrix cores, no residual step (ablation) */
  FX_PREC_ACE_FP16R = 8,  /* FP16 matrix cores on power-of-two-scaled operands + one FP64-combined residual step */
  FX_PREC_ACE_FP16 = 9    /* FP16 matrix cores on scaled operands, no residual step (ablation) */
} fx_prec;

/* Orthorhombic cell: grid n[0] x n[1] x n[2] (x, y, z), edges len[] in bohr. */
typedef struct fx_cell {
  int32_t n[3];
  double len[3];
} fx_cell;

/* kind: fx_kernel_kind; omega: screening parameter (bohr^-1, FX_HSE only);
 * scale: multiplies K (the mixing fraction alpha; 1 for the bare operator). */
typedef struct fx_kernel {
  int32_t kind;
  double omega;
  double scale;
} fx_kernel;

typedef struct fx_ctx fx_ctx;
typedef struct fx_ace fx_ace;
typedef struct fx_server fx_server;

/* Open a context on HIP device `device`.  hbm_budget_bytes caps the memory the
 * context may allocate (0 = 90% of the device's free memory).  *ctx receives
 * the handle.  Errors: FX_ERR_INVALID (ctx NULL), FX_ERR_DEVICE. */
fx_status fx_init(int device, size_t hbm_budget_bytes, fx_ctx** ctx);

/* Wait for the context's work, free everything it owns, destroy it.  ACE
 * handles and servers created on the context and still alive give their device
 * memory back here; afterwards fx_ace_free / fx_serve_destroy on them only
 * delete the handle, and every other call on them fails with FX_ERR_INVALID. */
fx_status fx_finalize(fx_ctx* ctx);

/* Text of the last error raised on the calling thread ("" if none). */
const char* fx_last_error(void);

/* Library version string. */
const char* fx_version(void);

/* Bytes currently allocated by the context, and the peak so far. */
fx_status fx_memory(const fx_ctx* ctx, size_t* in_use, size_t* peak);

/*
 * out = V_X[psi] phi   (Eq. applyVX; one Poisson-like solve per pair (j,k)).
 *
 * psi:  device, n_psi orbitals, column stride ld_psi (elements), dtype in_dtype.
 * phi:  device, n_phi targets, column stride ld_phi, dtype in_dtype; may be
 *       the same pointer as psi (then phi_k = psi_k for k < n_phi).
 * out:  device, n_phi columns, stride ld_out, dtype out_dtype; overwritten.
 * prec: FX_PREC_FP64, FX_PREC_FP32 or FX_PREC_FP32_ACC64.  The j-sum runs in
 *       ascending j in the accumulation precision, so results are bitwise
 *       repeatable and independent of how the pairs are batched.
 * When phi == psi with n_phi == n_psi and ld_phi == ld_psi on a cubic grid of
 *       edge 24, 48, 72 or 96, each unordered pair is solved once (the kernel
 *       is real and even, so the (k,j) solve is the conjugate of the (j,k)
 *       one): N(N+1)/2 solves instead of N^2.  Term j of column k is then taken
 *       from the solve of (min(j,k), max(j,k)); the result is still bitwise
 *       repeatable and batch-independent, and equals the full form up to
 *       rounding.
 * ex_energy_dev: optional device double receiving E_X = 1/2 Re sum_k
 *       <psi_k, out_k>; only allowed when phi == psi and ld_phi == ld_psi.
 * Errors: FX_ERR_INVALID, FX_ERR_UNSUPPORTED, FX_ERR_OOM, FX_ERR_DEVICE.
 */
fx_status fx_apply_vx(fx_ctx* ctx, const fx_cell* cell, const fx_kernel* kernel,
                      const void* psi, int32_t n_psi, int64_t ld_psi,
                      const void* phi, int32_t n_phi, int64_t ld_phi,
                      void* out, int64_t ld_out,
                      fx_dtype in_dtype, fx_dtype out_dtype, fx_prec prec,
                      void* stream, double* ex_energy_dev);

/* Size of the fixed device scratch region of fx_apply_vx_noalloc (per device). */
#define FX_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)

/*
 * fx_apply_vx without any device allocation, for callers that cannot
 * allocate: code under HIP graph capture, serving loops that must not call
 * hipMalloc, harnesses that forbid it.  Same arguments, layout, ownership,
 * result and errors as fx_apply_vx, with these differences:
 * - Everything beyond psi, phi and out (the grid tables, which it builds on
 *   the device, the pair work volume, partial sums, energy partials) lives in
 *   a file-scope device array of FX_NOALLOC_SCRATCH_BYTES that each device
 *   holds from the library's load until the process ends; fx_init looks up
 *   its address.  The call never allocates or frees device memory and never
 *   waits on the host.  A call whose tables and one pair volume (N_r complex
 *   values of the compute precision), plus partial sums when they cannot
 *   live in out, exceed the region fails with FX_ERR_INVALID before anything
 *   is launched; pass out in the accumulation type (complex128 for FP64 and
 *   FP32_ACC64, complex64 for FP32) so that partial sums live there.
 * - in_dtype must be the compute type (complex128 for FX_PREC_FP64, complex64
 *   for the FP32 forms): no conversion (FX_ERR_UNSUPPORTED otherwise).
 * - Each pair is solved as (j, k) even when phi == psi (no halving), and the
 *   j-sum of each target is one running sum (no sum groups, whatever the
 *   configuration's c_split); the result agrees with fx_apply_vx to rounding.
 * - All calls on one device share its region and its contents persist from
 *   call to call; calls that overlap in time on one device (other streams,
 *   threads or contexts) race and must be serialised by the caller.
 */
fx_status fx_apply_vx_noalloc(fx_ctx* ctx, const fx_cell* cell, const fx_kernel* kernel,
                              const void* psi, int32_t n_psi, int64_t ld_psi,
                              const void* phi, int32_t n_phi, int64_t ld_phi,
                              void* out, int64_t ld_out,
                              fx_dtype in_dtype, fx_dtype out_dtype, fx_prec prec,
                              void* stream, double* ex_energy_dev);

/*
 * Launch configuration of the V_X pair path for one grid, one V_X precision
 * and one form (phi == psi with all N targets, or not).  The batching of pair
 * solves into launches is the paper's batched-FFT step (Sec. 3.2); the
 * choices below are this library's.  Zero (or -1 where stated) means
 * automatic.  A configuration changes speed and rounding only: results stay
 * within the precision's tolerance (other kernel instantiations may fuse
 * multiply-adds differently), and are bitwise the same for every work_mb.
 */
typedef struct fx_vx_config {
  int32_t kernels;     /* 1 compile-time-specialised (cubic grids of edge 24, 48, 72, 96), 2 generic */
  int32_t work_mb;     /* pair work volume per batch, MiB (automatic: 8192, at most budget/4) */
  int32_t a_prefetch;  /* specialised plane-forward pass: 1 prefetch the next plane into
                          registers, 0 two workgroups per CU instead, -1 automatic (0) */
  int32_t b_variant;   /* specialised z pass x-tile: 1 the edge's default, 2 half of it,
                          3 whole x rows, 4 a persistent kernel (one y per workgroup,
                          the next tile's loads issued ahead) with whole x rows where
                          they fit the LDS (else the default tile); 0 automatic (4 at
                          edge 96, 3 at 72, else 1) */
  int32_t c_variant;   /* specialised plane-inverse pass: 1 the edge's default threads,
                          2 a larger count (fewer accumulators per thread, more waves),
                          3 and 4: 2 and 1 with the next work plane copied into LDS
                          while the current one is transformed (where two planes fit
                          the LDS: not FP64 at 72 and 96, which run 2 and 1 instead),
                          5: 2 with the inverse x transform across the lanes of a
                          wave (edges 72 and 96; elsewhere 2);
                          0 automatic (5 at edges 96 and 72, else 1) */
  int32_t a_variant;   /* specialised plane-forward pass threads: 1 the edge's default,
                          2 a count that divides the butterflies evenly, 3: 2 with the
                          product formed in a wave-level x transform (edges 72 and 96;
                          elsewhere 2); 0 automatic (3 for FP64 at edges 72 and 96,
                          else 1) */
  int32_t nt_hint;     /* specialised kernels: 1 read and write the pair volume with
                          non-temporal cache hints, 0 plain accesses, -1 automatic (1) */
  int32_t b_xtile;     /* generic z pass: x columns per workgroup */
  int32_t b_threads;   /* generic z pass: most threads per workgroup (64, 128, 192 or 256) */
  int32_t radix[3][4]; /* generic: radix schedule of each axis (x, y, z), stages in
                          order, 0-terminated; radices from {2,3,4,6,8,9,12} with
                          product n; an all-zero row is the default schedule */
  int32_t c_split;     /* specialised plane-inverse pass: S sum groups per target (1, 2,
                          4 or 8; 0 automatic = 1).  The terms of orbital j go to group
                          j mod S, each group summed in ascending j, the groups added in
                          order at the end: S times the pass's work items for calls with
                          few targets, at S partial sums per target of device memory.
                          The result depends on S (rounding) but not on the batch size
                          or on which targets share a launch */
} fx_vx_config;

/*
 * Autotuner: times candidate configurations for V_X applies of this shape
 * (n_psi orbitals, n_phi targets, phi_is_psi != 0 for the phi == psi form)
 * on synthetic data it allocates itself, by coordinate descent over the
 * fields above (kernel family; for the specialised kernels the prefetch form,
 * the z-pass tile, the plane-inverse and plane-forward threads and forms, the
 * cache hints and the plane-inverse sum groups; for the generic kernels the
 * radix schedule of each
 * axis, the z-pass tile and threads; then the batch volume), and stores the
 * fastest in the context, where every later fx_apply_vx, fx_build_ace and
 * served request of that grid, precision and form uses it.  Each candidate
 * is timed on a probe of at most ~2 full batches of pairs with HIP events on
 * `stream`; the call waits for the device.  *best (nullable) receives the
 * winner and *best_ms_per_kpair (nullable) its time per 1000 logical pairs
 * (j, k) of the probe.  The context's workspace is released at the end (the
 * candidates grew it to the largest batch tried): graphs captured from this
 * context before must not be replayed afterwards.
 * Errors: FX_ERR_INVALID, FX_ERR_UNSUPPORTED, FX_ERR_OOM, FX_ERR_DEVICE.
 */
fx_status fx_vx_autotune(fx_ctx* ctx, const fx_cell* cell, const fx_kernel* kernel, int32_t n_psi, int32_t n_phi,
                         int32_t phi_is_psi, fx_prec prec, void* stream, fx_vx_config* best,
                         double* best_ms_per_kpair);

/* Store `cfg` as the context's configuration for (grid, prec, form); NULL
 * clears it.  Errors: FX_ERR_INVALID (a field out of range, a radix schedule
 * that does not multiply to its edge, specialised kernels on another grid). */
fx_status fx_vx_set_config(fx_ctx* ctx, const fx_cell* cell, fx_prec prec, int32_t phi_is_psi,
                           const fx_vx_config* cfg);

/* The stored configuration for (grid, prec, form): *is_set = 1 and *cfg, or
 * *is_set = 0 and an all-automatic *cfg. */
fx_status fx_vx_get_config(fx_ctx* ctx, const fx_cell* cell, fx_prec prec, int32_t phi_is_psi, fx_vx_config* cfg,
                           int32_t* is_set);

/* Save the context's launch configurations to a text file, or load those of
 * this kind of device (architecture and CU count) from one (*n_loaded: how
 * many; nullable).  Lines for other devices are kept on save.  With the
 * environment variable FX_TUNE_CACHE set to a path, fx_init loads that file
 * if it exists and fx_vx_autotune saves to it after tuning.  Errors:
 * FX_ERR_INVALID (NULL argument, unreadable or malformed file). */
fx_status fx_vx_load_configs(fx_ctx* ctx, const char* path, int32_t* n_loaded);
fx_status fx_vx_save_configs(fx_ctx* ctx, const char* path);

/* Replay cache for fx_apply_vx and fx_apply_ace (the batched launches of
 * Sec. 3.2 without their per-launch cost): with max_entries > 0, the first
 * call with a given set of arguments (pointers included) runs as usual and is
 * then captured into a HIP graph held by the context; later calls with the
 * same arguments replay that graph on their stream.  Inputs are read when the
 * graph runs, so new values in the same buffers give new results; any other
 * argument makes a new entry (least recently used ones are dropped).
 * Entries made before a workspace was reallocated or a launch configuration
 * changed are never replayed.  Calls whose stream is itself being captured
 * bypass the cache.  max_entries = 0 (the default) turns it off and frees
 * the graphs.  Waits for the device.  Errors: FX_ERR_INVALID, FX_ERR_DEVICE. */
fx_status fx_graph_cache(fx_ctx* ctx, int32_t max_entries);
fx_status fx_graph_cache_stats(fx_ctx* ctx, int64_t* hits, int64_t* misses, int32_t* entries);

/*
 * Build the ACE factors of V_X[psi]: W = V_X psi (with vx_prec), M = psi^H W in
 * FP64, Hermitised, FP64 Cholesky -M = L L^H, L^{-1} in FP64, xi = W L^{-H}.
 * The handle keeps xi (FP64) and, on first use, the split forms needed by
 * ace_prec.  ex_energy_dev (device, nullable): one double receiving
 * E_X = 1/2 tr M, written on `stream` before the call returns.
 * Waits on `stream` once (Cholesky status).  Errors: FX_ERR_INVALID,
 * FX_ERR_UNSUPPORTED, FX_ERR_OOM, FX_ERR_NOT_POSDEF (-M not positive
 * definite: e.g. a single constant orbital with the Coulomb kernel),
 * FX_ERR_DEVICE.
 */
fx_status fx_build_ace(fx_ctx* ctx, const fx_cell* cell, const fx_kernel* kernel,
                       const void* psi, int32_t n_psi, int64_t ld_psi, fx_dtype in_dtype,
                       fx_prec vx_prec, fx_prec ace_prec, void* stream,
                       fx_ace** ace, double* ex_energy_dev);

/*
 * out = K_ACE phi = -xi (xi^H phi).  prec: one of the FX_PREC_ACE_* values.
 * The low-precision forms split each operand X into round(X) and
 * round(X - round(X)) and add the three products that matter in FP64; the
 * FP16 forms first scale xi, each column of phi and each column of xi^H phi
 * by powers of two (largest magnitude in [2^13, 2^14)) and divide the
 * factors out exactly.  Error against FP64 (96^3, N = R = 1024, element-wise):
 * FP32 + residual 3e-6, BF16 + residual 7e-6 (floor about 1e-5), FP16 +
 * residual 1.3e-6.
 * phi: device, n_phi columns of N_r, stride ld_phi, dtype in_dtype.
 * out: device, n_phi columns, stride ld_out, dtype out_dtype; overwritten.
 * The first call with a new precision or a larger n_phi allocates; later
 * calls do not.  Errors: FX_ERR_INVALID, FX_ERR_UNSUPPORTED, FX_ERR_OOM,
 * FX_ERR_DEVICE.
 */
fx_status fx_apply_ace(fx_ctx* ctx, const fx_ace* ace,
                       const void* phi, int32_t n_phi, int64_t ld_phi,
                       void* out, int64_t ld_out,
                       fx_dtype in_dtype, fx_dtype out_dtype, fx_prec prec, void* stream);

/* Copy the FP64 factors out of a handle (device pointers, caller-owned):
 * xi (N_r x N, ld = N_r, c128), L (N x N column-major, c128), M likewise.
 * Any pointer may be NULL.  Synchronous. */
fx_status fx_ace_export(const fx_ace* ace, void* xi, void* L, void* M);

/* Number of orbitals and grid points of a handle. */
fx_status fx_ace_shape(const fx_ace* ace, int32_t* n, int64_t* n_r);

/* Free an ACE handle (waits for its work first).  Valid before or after
 * fx_finalize of its context (after it, only the handle is left to delete). */
fx_status fx_ace_free(fx_ace* ace);

/*
 * End-of-step operations of PT-CN (all arithmetic FP64; complex64 blocks are
 * widened on input and rounded on output).
 *
 * fx_apply_kinetic: out = T phi with T = -(1/2) Laplacian, the kinetic term of
 *   the Hamiltonian (Sec. 2), on the periodic grid of the cell: each planewave
 *   coefficient of phi_k is multiplied by |G|^2/2, G_a = 2 pi m_a / len_a with
 *   m_a in FFT order (on an even edge the row m_a = n_a/2 has |G_a| =
 *   pi n_a / len_a).  phi: device, n_phi columns of N_r, stride ld_phi,
 *   in_dtype; out: device, n_phi columns, stride ld_out, out_dtype,
 *   overwritten, must not overlap phi.  Computed by the V_X pair path (FP64)
 *   with the constant orbital 1 and the kernel |G|^2/(2 N_r); the first call
 *   on a grid allocates its tables and workspace.  Errors: FX_ERR_INVALID,
 *   FX_ERR_UNSUPPORTED, FX_ERR_OOM, FX_ERR_DEVICE.
 *
 * fx_pt_residual: the residual of the PT-CN fixed point (the residual
 *   algorithm of Sec. 3.3, for the parallel-transport equation of Sec. 2):
 *     S = Psi^H (H Psi),  R = Psi + (i dt/2)(H Psi - Psi S) - Psi_half.
 *   psi, hpsi, psi_half: device blocks of n columns, stride ld, dtype; hpsi
 *   NULL means H = V_X[psi] (computed by the pair path with vx_prec; kernel
 *   then required).  kinetic nonzero adds the kinetic term: H Psi becomes
 *   hpsi + T psi (or V_X[psi] psi + T psi), T as in fx_apply_kinetic.
 *   r_out: device, n columns, stride ld_r, dtype; must not overlap the
 *   inputs.  s_out: nullable device n x n complex128 column-major, receives
 *   S.  The cell gives N_r (and the grid and lengths when hpsi is NULL or
 *   kinetic is set).  Errors: FX_ERR_INVALID, FX_ERR_UNSUPPORTED, FX_ERR_OOM,
 *   FX_ERR_DEVICE.
 *
 * fx_orthonormalize: Cholesky-QR re-orthonormalisation in place (Sec. 3.4):
 *   S = Psi^H Psi, S = L L^H, Psi <- Psi L^{-H}.  Waits on `stream` once (the
 *   Cholesky status); FX_ERR_NOT_POSDEF if the columns are linearly dependent.
 *
 * fx_density: rho(r) = sum_i f_i |psi_i(r)|^2 (Sec. 3.4), summed over i in
 *   ascending order in FP64.  occ: nullable device array of n doubles (all 1
 *   if NULL); rho: device array of nr doubles, overwritten.
 */
fx_status fx_apply_kinetic(fx_ctx* ctx, const fx_cell* cell, const void* phi, int32_t n_phi, int64_t ld_phi,
                           void* out, int64_t ld_out, fx_dtype in_dtype, fx_dtype out_dtype, void* stream);
fx_status fx_pt_residual(fx_ctx* ctx, const fx_cell* cell, const fx_kernel* kernel, const void* psi,
                         const void* hpsi, const void* psi_half, int32_t n, int64_t ld, fx_dtype dtype,
                         double dt, fx_prec vx_prec, int32_t kinetic, void* r_out, int64_t ld_r, void* s_out,
                         void* stream);
fx_status fx_orthonormalize(fx_ctx* ctx, void* psi, int32_t n, int64_t ld, int64_t nr, fx_dtype dtype,
                            void* stream);
fx_status fx_density(fx_ctx* ctx, const void* psi, int32_t n, int64_t ld, int64_t nr, fx_dtype dtype,
                     const double* occ, double* rho, void* stream);

/*
 * Serving: continuous batching of V_X / ACE requests over resident orbitals.
 *
 * fx_serve_create: batches run on n_streams streams, at most one per stream at
 *   a time (a batch waits in the host queue rather than behind another
 *   stream's batch); max_slots bounds the workspaces kept for them (slot i
 *   uses stream i mod n_streams).  Waiting requests of one operation are
 *   merged into one launch of up to max_batch_pairs pairs: K_ACE requests of
 *   one trajectory; V_X requests of up to eight trajectories that share the
 *   grid (edge 24, 48, 72 or 96), cell lengths, kernel, orbital count, dtype
 *   and precision (orbitals in the compute type), each target paired with
 *   its own trajectory's orbitals (V_X requests on other grids merge within
 *   their trajectory).  Results do not depend on the merge.  Admission keeps
 *   the memory of resident trajectories plus in-flight requests within
 *   hbm_budget_bytes (0 = the context budget): a batch that cannot fit even
 *   with every slot idle is refused with FX_ERR_OOM; an arrival that finds
 *   max_queue requests already waiting is refused with FX_ERR_BUSY (0 = no
 *   limit).
 * fx_serve_register: copy psi (N_r x n, dtype) into library-owned resident
 *   memory as trajectory `traj`, and build its ACE factors (ace_prec).
 * fx_serve: replay `n_reqs` requests whose arrival times (seconds from the
 *   start) are t_arrival_s; request i computes V_X (op 0) or K_ACE (op 1)
 *   applied to orbitals first..first+count-1 of its trajectory, written to
 *   its `out` (device, ld_out, dtype of the trajectory).  Returns when every
 *   request has finished; per_req_status/per_req_latency_ms (nullable host
 *   arrays of n_reqs) receive each request's status and latency (completion
 *   time minus arrival time), and report the aggregate.  Statuses: FX_OK,
 *   FX_ERR_INVALID (unknown trajectory or operation, orbitals out of range,
 *   NULL out), FX_ERR_OOM, FX_ERR_BUSY, FX_ERR_CANCELLED (cancelled, or not
 *   reached because the loop stopped on a device error).
 * fx_serve_cancel: cancel request `request` (an index into the request array
 *   of the fx_serve call running on this server, or of the next call if none
 *   is running); callable from another thread while fx_serve runs.  A
 *   request not yet dispatched is dropped with FX_ERR_CANCELLED; one already
 *   on the device completes normally.  Cancellations are forgotten when
 *   fx_serve returns.
 */
typedef struct fx_serve_cfg {
  int32_t max_slots;
  int32_t n_streams;
  int32_t max_batch_pairs;
  size_t hbm_budget_bytes;
  int32_t autotune;   /* nonzero: fx_serve_register runs fx_vx_autotune for the trajectory's
                         grid and V_X precision (requests of autotune_targets targets against
                         its n orbitals) and for its ACE build (phi == psi), unless the context
                         already holds configurations for them */
  int32_t autotune_targets; /* targets per V_X request the tuning assumes (0 = 8) */
  int32_t vx_work_mb;  /* pair work volume per launch of a served V_X batch, MiB (0 = 1024):
                          short launches let requests on other streams interleave */
  int32_t max_queue;   /* waiting requests beyond which arrivals get FX_ERR_BUSY (0 = no limit) */
} fx_serve_cfg;

typedef struct fx_request {
  int32_t traj;
  int32_t op; /* 0 = V_X, 1 = ACE */
  int32_t first;
  int32_t count;
  double t_arrival_s;
  void* out;
  int64_t ld_out;
} fx_request;

typedef struct fx_serve_report {
  double p50_ms, p99_ms, mean_ms, max_ms;
  double req_per_s, pairs_per_s, busy_frac, wall_s;
  int64_t n_done, n_rejected, n_batches; /* n_rejected: FX_ERR_OOM and FX_ERR_BUSY */
  size_t hbm_peak_bytes;
  int64_t n_cancelled;
} fx_serve_report;

fx_status fx_serve_create(fx_ctx* ctx, const fx_serve_cfg* cfg, fx_server** srv);
fx_status fx_serve_register(fx_server* srv, int32_t traj, const fx_cell* cell, const fx_kernel* kernel,
                            const void* psi, int32_t n, int64_t ld, fx_dtype dtype,
                            fx_prec vx_prec, fx_prec ace_prec);
fx_status fx_serve(fx_server* srv, const fx_request* reqs, int32_t n_reqs,
                   fx_status* per_req_status, double* per_req_latency_ms, fx_serve_report* report);
fx_status fx_serve_cancel(fx_server* srv, int32_t request);
/* Release a server: its resident orbitals, ACE factors, workspaces and streams
 * (after waiting for the device), and the context budget it capped.  Valid
 * before or after fx_finalize of its context. */
fx_status fx_serve_destroy(fx_server* srv);

#ifdef __cplusplus
}
#endif

#endif /* LIBFOCK_FOCK_H */
