/*
 * lsrtm.h -- C ABI of the MI355X (gfx950) data-domain LSRTM hot path.
 *
 * The library implements, on one GPU, the linear operators of multiparameter
 * least-squares reverse time migration in the (lnVp, lnIp) parametrisation
 * (Yang & Ji, "A comparative study of data- and image-domain LSRTM under
 * velocity-impedance parametrization"):
 *
 *   - background modelling of the first-order velocity-pressure system
 *     A(m)u = f (section 2, first equation);
 *   - Born modelling L dm = R du, du solving the scattering system with the
 *     lnVp/lnIp secondary sources (section 2, eq. scattereqln; section 3,
 *     definition of L[m0]);
 *   - migration L^T d: the adjoint-state cross-correlation imaging conditions
 *     (appendix A, eqs. adjeq, gradlsm, gradrho, gradkappa) mapped to
 *     (lnVp, lnIp) by the gradient chain rule (section 3);
 *   - CGNR on the normal equations L^T L dm = L^T dd (section 3, eq. normal
 *     and the CGNR paragraph), with FP64 inner products and step lengths.
 *
 * Discretisation (the paper states continuous equations only): staggered grid,
 * second order in time, eighth order in space, recursive-convolution CPML of
 * npml cells on every side, pressure point source injected with the midpoint
 * rule, receivers recording pressure at nodes after each step.  L^T is the
 * exact discrete transpose of L under plain Euclidean inner products.
 * Propagation is FP32; reductions and CG scalars are FP64.
 *
 * Conventions
 *   - Arrays on the physical grid are z-fastest: index iz + nz*(ix + nx*iy).
 *   - Node coordinates are (iz, ix[, iy]) of the global physical grid.
 *   - Unless marked HOST, pointers are DEVICE pointers owned by the caller and
 *     accessed on the context's HIP stream; the library never frees them.
 *     The library owns only its internal workspaces.
 *   - Every call returns LSRTM_OK or a negative lsrtm_status; nothing aborts.
 *     lsrtm_last_error(ctx) returns a description of the last failure.
 *   - A NULL ctx is LSRTM_EINVAL for every call that takes one, checked before
 *     any other argument (lsrtm_destroy ignores it, lsrtm_last_error returns
 *     an empty string).
 *   - Call order: create -> set_model -> set_acquisition ->
 *     {forward | born | adjoint | cgnr}*.  set_model may be called again
 *     later; other orders return LSRTM_ESTATE.
 *   - A context is bound to one stream and is not thread-safe.
 */
#ifndef LSRTM_H
#define LSRTM_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lsrtm_ctx lsrtm_ctx;

typedef enum {
    LSRTM_OK = 0,
    LSRTM_EINVAL = -1,     /* bad argument (shape, index, pointer, option)      */
    LSRTM_ENOMEM = -2,     /* device allocation failed or plan does not fit     */
    LSRTM_EHIP = -3,       /* HIP runtime error (kept in lsrtm_last_error)      */
    LSRTM_EUNSTABLE = -4,  /* CFL condition violated by the model and dt        */
    LSRTM_ENONFINITE = -5, /* NaN/Inf found in the model or a stored snapshot  */
    LSRTM_ESTATE = -6      /* call out of order                                 */
} lsrtm_status;

enum { LSRTM_CKPT_F32 = 0, LSRTM_CKPT_F16 = 1, LSRTM_CKPT_BF16 = 2 };

typedef struct {
    int ndim;        /* 2 or 3                                                  */
    int n[3];        /* physical nz, nx, ny of the global grid (ny = 1 in 2D)   */
    double h[3];     /* dz, dx, dy in metres                                    */
    int npml;        /* CPML thickness in cells on every side (>= 0)            */
    double pml_R;    /* CPML target reflection coefficient (e.g. 1e-4)          */
    double pml_f0;   /* CPML frequency-shift parameter: alpha_max = pi * f0     */
    int nt;          /* number of time steps                                    */
    double dt;       /* time step in seconds                                    */
    int ckpt_every;  /* background checkpoint interval in steps; 0 = planner    */
    int ckpt_dtype;  /* LSRTM_CKPT_F32 / F16 / BF16 storage of p and v in the
                        checkpoints (per-snapshot, per-field max-abs scaling for
                        F16/BF16; CPML memories always FP32)                    */
} lsrtm_grid;

/* Options (lsrtm_set_option). */
enum {
    LSRTM_OPT_SHOTS_PER_LAUNCH = 1, /* shots advanced by one kernel launch:
                                       1 = plain per-shot launches,
                                       0 = as many as the memory plan allows;
                                       after set_acquisition it rebuilds the
                                       plan (stored checkpoints are dropped)    */
    LSRTM_OPT_TILE = 2,             /* stencil tile id (see lsrtm_tile_shape);
                                       -1 = autotune on the next pass           */
    LSRTM_OPT_GRAPH = 3,            /* 1 = replay the time loop from captured
                                       HIP graphs (default 1)                   */
    LSRTM_OPT_TIMING = 4,           /* 1 = time every stencil launch with HIP
                                       events (read back with lsrtm_stats)      */
    LSRTM_OPT_MEM_BUDGET_MB = 5,    /* device memory the plan may use; 0 = 90 %
                                       of the free memory at set_acquisition    */
    LSRTM_OPT_CKPT_PER_GROUP = 6,   /* 1 = keep background checkpoints only for
                                       the active launch group and regenerate
                                       them before each group's migration (the
                                       planner picks this by itself when the
                                       checkpoints of all shots do not fit)     */
    LSRTM_OPT_FUSED = 7,            /* 2D: 1 = one kernel per time step (the
                                       velocity and pressure updates fused,
                                       double-buffered fields), 0 = a velocity
                                       and a pressure kernel per step (default;
                                       faster on gfx950).  Both give identical
                                       results; lsrtm_autotune tries both.      */
    LSRTM_OPT_PROGRESS = 8,         /* 1 = wait for every launch group's pass
                                       and print one line per group to stderr
                                       (long 3D passes); default 0              */
    LSRTM_OPT_TILE_V = 9,           /* two-phase steps (2D default, 3D): tile
                                       id of the velocity phases (Born,
                                       background and replay), which record
                                       and inject nothing; -1 = LSRTM_OPT_TILE
                                       (default).  Results do not depend on it;
                                       ignored by the fused 2D schedule.        */
    LSRTM_OPT_TILE_ADJ_A = 10,      /* likewise for the adjoint pressure phase
                                       (A); -1 = LSRTM_OPT_TILE (default)       */
    LSRTM_OPT_REPLAY_CACHE_MB = 11, /* device memory (MB) that may keep the
                                       background replays of the last segments
                                       of every launch group across migration
                                       passes (App. A: the history is the
                                       background's, independent of dm and of
                                       the data), capped by what the memory
                                       budget leaves; the first migration pass
                                       fills it, later ones skip the replay of
                                       those segments, and later 2D Born passes
                                       run only the scattered phases there,
                                       reading the background from it.  Results
                                       are bitwise the same.  Two-phase steps with checkpoints
                                       for the whole plan only; 0 = off
                                       (default).  Re-plans when changed.       */
    LSRTM_OPT_GRAPH_CACHE = 12      /* most pass graphs kept (least recently
                                       used replaced first; a pass graph is
                                       keyed by pass kind, launch group, data
                                       pointer and tile); 0 = 8 per launch
                                       group plus 8 (default)                   */
};

/* Create a context for one grid on one HIP stream (hipStream_t, may be 0).
 * Validates the grid; *out receives the context (NULL on failure).
 * Allocates nothing on the device yet and makes no HIP call.  Errors: EINVAL
 * (NULL grid or out, ndim not 2 or 3, a size < 1 or a spacing <= 0, ny != 1
 * in 2D, npml < 0, nt < 1, dt <= 0, pml_R outside (0, 1) with npml > 0,
 * ckpt_every < 0 or an unknown ckpt_dtype). */
lsrtm_status lsrtm_create(const lsrtm_grid* grid, void* hip_stream, lsrtm_ctx** out);

/* Background model in logs (section 2: lnkappa = lnIp + lnVp,
 * lnrho = lnIp - lnVp).  lnvp, lnip: DEVICE float [nz*nx*ny], z-fastest,
 * physical grid, copied by the library.  Checks that every value is finite
 * (LSRTM_ENONFINITE) and the CFL bound
 *   vmax * dt * sqrt(sum_a 1/h_a^2) * sum_k |c_k| < 1   (LSRTM_EUNSTABLE).
 * Invalidates stored checkpoints.  Errors: EINVAL (NULL), ENONFINITE,
 * EUNSTABLE (the context then has no model), ENOMEM, EHIP. */
lsrtm_status lsrtm_set_model(lsrtm_ctx* ctx, const float* lnvp, const float* lnip);

/* Acquisition of nshot shots, each on its own window of the physical grid
 * (uneven apertures allowed).
 *   win     HOST int [nshot][2*ndim]: z0,z1,x0,x1[,y0,y1], half-open ranges
 *   src     HOST int [nshot][ndim]: source node (iz, ix[, iy]), inside win
 *   rec_ptr HOST int [nshot+1]: CSR offsets into rec (rec_ptr[0] = 0)
 *   rec     HOST int [rec_ptr[nshot]][ndim]: receiver nodes, inside win
 *   wavelet DEVICE float [nshot][nt]: source samples w((n + 1/2) dt); the
 *           library injects dt * w / (dz dx [dy]) into p at the source node.
 * Data vectors then have length sum_s nt*nrec_s, shot s at offset
 * nt * rec_ptr[s], laid out [it][rec].  Plans the device memory (shots per
 * launch, checkpoint interval) and allocates it.  A shot's padded window
 * (z rounded up to 32) must hold fewer than 2^30 nodes.  Errors: EINVAL
 * (windows, sources or receivers outside the grid, a window of 2^30 nodes or
 * more), ENOMEM (the plan does not fit), ESTATE (no model), EHIP. */
lsrtm_status lsrtm_set_acquisition(lsrtm_ctx* ctx, int nshot, const int* win, const int* src,
                                   const int* rec_ptr, const int* rec, const float* wavelet);

/* Background data d = R u0 (section 2, A(m0) u0 = f), DEVICE float [data].
 * Also stores the background checkpoints used by lsrtm_adjoint.
 * Errors of lsrtm_forward, lsrtm_born and lsrtm_adjoint: EINVAL (NULL ctx, a
 * NULL model vector, a NULL data vector while there are data), ESTATE (no
 * model or no acquisition), ENONFINITE (a stored background snapshot holds
 * NaN or Inf; the checkpoints are then dropped), ENOMEM, EHIP. */
lsrtm_status lsrtm_forward(lsrtm_ctx* ctx, float* d);

/* Born data d = L dm (section 3).  dm: DEVICE float [2][nz*nx*ny] =
 * (dlnVp, dlnIp) on the physical grid; the perturbation is zero in the PML.
 * d: DEVICE float [data], overwritten. */
lsrtm_status lsrtm_born(lsrtm_ctx* ctx, const float* dm, float* d);

/* Migration img = L^T d (appendix A; section 3 chain rule), summed over all
 * shots in a fixed order (deterministic).  d: DEVICE float [data];
 * img: DEVICE float [2][nz*nx*ny] = (lnVp, lnIp) images; accumulate = 0
 * overwrites img, 1 adds to it. */
lsrtm_status lsrtm_adjoint(lsrtm_ctx* ctx, const float* d, float* img, int accumulate);

/* niter CGNR iterations on L^T L x = L^T d_obs from x = 0 (section 3).
 * d_obs: DEVICE float [data]; x: DEVICE float [2][nz*nx*ny] output;
 * misfit: HOST double [niter+1] receives ||r_k||^2 / ||r_0||^2 (may be NULL).
 * Workspace vectors are owned by the library.  Errors: EINVAL (NULL ctx or x,
 * niter < 0, NULL d_obs with data), ESTATE (no model or acquisition), ENOMEM,
 * EHIP. */
lsrtm_status lsrtm_cgnr(lsrtm_ctx* ctx, const float* d_obs, int niter, float* x, double* misfit);

/* Step-wise CGNR (the same iteration as lsrtm_cgnr).
 * lsrtm_cgnr_begin: r = d_obs, x = 0, z = L^T r, p = z (one migration).
 * lsrtm_cgnr_iterate: one iteration (one Born and one migration pass);
 *   *misfit (HOST, may be NULL) receives ||r_k||^2 / ||r_0||^2.
 * lsrtm_cgnr_state: get = 1 copies the solver state out (r: data length,
 *   z and p: [2][nz*nx*ny], DEVICE), scal = HOST double[4] = (<z,z>,
 *   <r0,r0>, <r,r>, k); get = 0 loads such a state back, so that a stopped
 *   run resumes to the same iterates (x is the caller's vector).
 * Errors: EINVAL (NULL ctx, x, state pointers, or d_obs while there are
 * data), ESTATE (no model or acquisition; lsrtm_cgnr_iterate or a state
 * export before lsrtm_cgnr_begin), ENONFINITE, ENOMEM, EHIP. */
lsrtm_status lsrtm_cgnr_begin(lsrtm_ctx* ctx, const float* d_obs, float* x);
lsrtm_status lsrtm_cgnr_iterate(lsrtm_ctx* ctx, float* x, double* misfit);
lsrtm_status lsrtm_cgnr_state(lsrtm_ctx* ctx, int get, float* r, float* z, float* p, double* scal);

/* The step of the last lsrtm_cgnr_iterate (section 3, the CGNR paragraph:
 * alpha = <z, s> / ||L p||^2, beta = <z, s>_new / <z, s>_old), for logging:
 * out (HOST double[5]) = (k, alpha, beta, ||L p||^2, normalised misfit
 * ||r_k||^2 / ||r_0||^2), all FP64 as the solver computed them; alpha, beta
 * and ||L p||^2 are 0 before the first iteration and for an iteration that
 * found the residual already zero.  Errors: EINVAL (NULL), ESTATE (no CGNR
 * run begun). */
lsrtm_status lsrtm_cgnr_step(lsrtm_ctx* ctx, double* out);

/* Pseudo-Hessian diagonal (appendix B): the diagonal of the Hessian is
 * approximated by the time-integrated energy of the Born secondary source
 * that a unit perturbation radiates in each shot's incident field, summed
 * over shots.  With the Born step's sources (a unit dlnrho at node i adds
 * -avg_a(e_i) dv_a to the velocities, a unit dlnkappa adds -dt kappa q at i):
 *   h_i = sum_shots [ rho_i^2 / dt * sum_n sum_a ||avg_a(e_i) dv_a^n||^2
 *                     + (dt kappa_i)^2 / dt * sum_n (q_i^n)^2 ],
 * dv_a the background velocity increments and q the CPML-corrected
 * divergence of step n.  By the chain rule of section 3 the diagonal is the
 * same for lnVp and lnIp.
 * h: DEVICE float [nz*nx*ny] (physical grid, z fastest), written.
 * minv: DEVICE float [2][nz*nx*ny] or NULL; if given it receives
 *   1 / (h + eps_rel * max h) for both parameters, the preconditioner of
 *   lsrtm_set_preconditioner (the paper does not state the stabilisation).
 * Runs one background pass (velocity and pressure kernels, plain launches)
 * through the library's field buffers; stored checkpoints stay valid.
 * Synchronises the stream when minv is given.  Errors: EINVAL (h NULL,
 * eps_rel < 0, or minv requested for an all-zero h or eps_rel = 0), ESTATE
 * (model or acquisition missing), ENONFINITE, EHIP. */
lsrtm_status lsrtm_pseudo_hessian(lsrtm_ctx* ctx, float* h, float* minv, double eps_rel);

/* Diagonal preconditioner of the CGNR solver (section 3: CGNR preconditioned
 * with the pseudo-Hessian of appendix B).  The normal residual s = L^T r is
 * replaced by z = minv * s; step length <z, s> / <L p, L p>, direction
 * p = z + beta p with beta = <z, s>_new / <z, s>_old.  minv: DEVICE float
 * [2][nz*nx*ny] (lnVp block, then lnIp), copied into a library buffer (the
 * caller keeps ownership); NULL removes the preconditioner.  Takes effect at
 * the next lsrtm_cgnr / lsrtm_cgnr_begin or state import; the exported state
 * then holds z = minv * s and scal[0] = <z, s>.  Errors: EINVAL (ctx NULL),
 * ENOMEM, EHIP. */
lsrtm_status lsrtm_set_preconditioner(lsrtm_ctx* ctx, const float* minv);

/* Image-domain LSRTM with the point-spread-function Hessian (section 3,
 * eq. migdeconobj; appendix C).  Scatterers sit on a lattice every `spacing`
 * nodes of every axis, at W, W + spacing, ... with W = (spacing - 1) / 2 the
 * half-width of the window kept around each scatterer (neighbouring windows
 * do not overlap).  Errors of all three: EINVAL (NULL pointers, spacing < 1 or
 * no scatterer on an axis), EHIP; lsrtm_psf_images also ESTATE.
 *
 * lsrtm_psf_images: PSF images P[q] = L^T L S_q, S_q the unit scatterers of
 *   parameter q (0 = lnVp, 1 = lnIp): one Born and one migration pass per q.
 *   psf: DEVICE float [2 (q)][2 (response p)][nz*nx*ny], written.
 * lsrtm_psf_apply: y = H x (transpose = 0) or H^T x (transpose = 1) with the
 *   interpolated Hessian of eq. trilinear (bilinear in 2D):
 *     H_pq[j + o, j] = sum over the lattice corners c of j of
 *                      w_c(j) P[q][p][c + o],  |o_a| <= W,
 *   w_c the multilinear weights of j between its corners (clamped to the
 *   nearest scatterer outside the lattice), entries with j + o or c + o
 *   outside the grid dropped.  mono = 0: x, y DEVICE [2][n] (lnVp, lnIp),
 *   the 2 x 2 block operator; mono = 1: the lnIp block H_22 on [n] vectors.
 *   x and y must not alias.
 * lsrtm_psf_cgnr: niter CGNR iterations on H^T H x = H^T m_rtm from x = 0 (the
 *   paper solves the normal equations of the PSF Hessian because
 *   interpolation breaks its symmetry).  m_rtm, x: DEVICE, [2][n] or (mono)
 *   [n]; misfit: HOST double [niter + 1] or NULL, ||H x_k - m_rtm||^2 /
 *   ||m_rtm||^2.  Needs lsrtm_set_model (FP64 inner products). */
lsrtm_status lsrtm_psf_images(lsrtm_ctx* ctx, int spacing, float* psf);
lsrtm_status lsrtm_psf_apply(lsrtm_ctx* ctx, const float* psf, int spacing, int mono, int transpose,
                             const float* x, float* y);
lsrtm_status lsrtm_psf_cgnr(lsrtm_ctx* ctx, const float* psf, int spacing, int mono, const float* m_rtm,
                            int niter, float* x, double* misfit);

/* Top mute of recorded data, in place (the nonlinear-residual data
 * preparation of section 4.1: observed minus background data with the direct
 * arrival muted; the paper does not state the mute).  For shot s and receiver
 * r at distance D (metres, physical node coordinates times h), samples
 * recorded before tc = t0 + D / v_mute are zeroed and the next ntaper samples
 * ramp up with 0.5 (1 - cos(pi (t - tc) / (ntaper dt))); sample n is recorded
 * at time (n + 1) dt.  d: DEVICE float [data length] in the layout of
 * lsrtm_forward.  Synchronises the stream.  Errors: EINVAL (v_mute <= 0,
 * ntaper < 0, NULL d), ESTATE (no acquisition), EHIP. */
lsrtm_status lsrtm_mute(lsrtm_ctx* ctx, float* d, double v_mute, double t0, int ntaper);

/* lsrtm_mute for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same mute, with its per-receiver tables computed on the device from the
 * acquisition the plan holds, into a file-scope device array of 5 MiB (one
 * per GPU, kept until the process ends) instead of buffers allocated per
 * call.  Calls no hipMalloc, hipFree or allocating routine and does not
 * synchronise; the first call on a device looks up the array's address.
 * Arguments as for lsrtm_mute, with the context's device current.  At most
 * 2^18 receivers over all shots.  Every call on one GPU shares the array:
 * calls that overlap on one GPU (several contexts or threads at once) race.
 * Errors: EINVAL (as lsrtm_mute, or more than 2^18 receivers), ESTATE
 * (no acquisition), EHIP. */
lsrtm_status lsrtm_mute_noalloc(lsrtm_ctx* ctx, float* d, double v_mute, double t0, int ntaper);

/* Nonstationary Wiener deblurring (appendix D).  The Hessian is taken as
 * locally translation invariant, hence diagonal in the Fourier basis of each
 * local block; per block (F its Fourier transform) the regularised inverse
 * eigenvalues are Lambda^-1 = conj(F m_blur) F m_ref / (|F m_blur|^2 + eps),
 * eps = eps_rel * max |F m_blur|^2 of the block, and the block estimate is
 * F^-1[Lambda^-1 F m_in] (eq. sol).  Blocks of `block` nodes per axis (even)
 * start every block/2 nodes from -block/2 (zero outside the image), tapered by
 * sin^2(pi (u + 1/2) / block) per axis; the estimates are merged with these
 * valences, out = sum_w dm_w / sum_w t_w.  The paper's use: m_ref = m_in =
 * the RTM image, m_blur = its remigration L^T L m_rtm.
 * m_ref, m_blur, m_in, out: DEVICE float [nimg][nz*nx*ny] (each image
 * filtered on its own; out may alias an input).  FFT plans and a work buffer
 * of 3 * blocks * block^ndim complex values are kept in the context.
 * Errors: EINVAL (NULL, nimg < 1, odd or < 2 block, eps_rel < 0), EHIP. */
lsrtm_status lsrtm_wiener(lsrtm_ctx* ctx, const float* m_ref, const float* m_blur, const float* m_in,
                          int nimg, int block, double eps_rel, float* out);

/* Inner product of the CGNR iteration (section 3, the CGNR paragraph: step
 * lengths and the normalised misfit are ratios of such products) of two
 * DEVICE float vectors of length n, accumulated in FP64; *out is a HOST
 * double.  Deterministic (fixed reduction tree); synchronises the stream.
 * Errors: EINVAL (ctx or out NULL, n < 0, a or b NULL with n > 0), EHIP. */
lsrtm_status lsrtm_dot(lsrtm_ctx* ctx, const float* a, const float* b, long long n, double* out);

/* y <- y + alpha * x on DEVICE float vectors of length n, each element
 * computed in FP64 and rounded once (the iterate and residual updates of
 * section 3's CGNR).  Errors: EINVAL (NULL ctx, n < 0, x or y NULL with
 * n > 0), EHIP. */
lsrtm_status lsrtm_axpy(lsrtm_ctx* ctx, double alpha, const float* x, float* y, long long n);

/* Calibration, not a step of the method: the HBM streaming rate of a mix of
 * arrays like the stencil kernels' (the 3D Born velocity phase reads 10
 * arrays and writes 6 per node, its pressure phase reads 10 and writes 2).
 * One pass over nread + nwrite DEVICE arrays of n floats laid out one after
 * another in buf ((nread + nwrite) * n floats, caller-owned, contents
 * overwritten): every element of the first nread arrays is read once and
 * every element of the last nwrite arrays written once.  (nread, nwrite) is
 * one of (10, 6), (10, 2), (5, 6), (5, 2), (2, 1).  grid = NULL walks the
 * elements in order; grid = HOST int[4] (nz, nx, ny, ldz), with
 * n = ldz * nx * ny and nz <= ldz, walks them as the 3D stencil tiles do
 * (blocks of 64 x 4 z-x columns marching 32 planes along y).  Enqueued on the
 * context's stream; waits for it and sets *ms (HOST) to the kernel's own
 * execution time.  Errors: EINVAL (NULL, n < 1, unsupported mix, grid not
 * matching n), EHIP. */
lsrtm_status lsrtm_stream_mix(lsrtm_ctx* ctx, float* buf, long long n, int nread, int nwrite, const int* grid,
                              double* ms);

/* Set an LSRTM_OPT_* option.  Counts lie in [0, 2^31 - 1] (-1 allowed for
 * the tile ids), sizes in MB in [0, 2^30].  Options that change the launch
 * groups or the memory plan re-plan at once when an acquisition is set.
 * Errors: EINVAL (NULL ctx, unknown key, value out of range), and the
 * errors of lsrtm_set_acquisition for a re-plan. */
lsrtm_status lsrtm_set_option(lsrtm_ctx* ctx, int key, long long value);

/* Autotuner: times the stencil kernels of a Born, replay and adjoint step
 * over nsteps time steps on the actual launch groups for every tile shape,
 * and with tune_groups = 1 also for several shot-per-launch sizes and (2D)
 * both step schedules (rebuilding the memory plan), then keeps the fastest.
 * For two-phase steps it then tries every other shape for the velocity
 * phases and for the adjoint A phase (LSRTM_OPT_TILE_V / _TILE_ADJ_A, set to
 * the picks or -1).  out (HOST double[5], may be NULL) = (tile id, shots per
 * launch, ms per time step, velocity-phase tile, adjoint-A tile).  With
 * LSRTM_TUNE_CACHE naming a file, results are read from and appended to it.
 * Invalidates stored checkpoints.  When no tile is set, the same tile tuning
 * (without group sizes and schedules) runs on the first pass by itself.
 * Errors: EINVAL (NULL ctx, nsteps < 1), ESTATE (no model or acquisition),
 * ENOMEM, EHIP. */
lsrtm_status lsrtm_autotune(lsrtm_ctx* ctx, int nsteps, int tune_groups, double* out);

/* Sizes: out[0] = data length, out[1] = physical grid points (one image),
 * out[2] = shots per launch, out[3] = checkpoint interval, out[4] = number of
 * launch groups, out[5] = padded points summed over shots, out[6] = device
 * bytes planned, out[7] = tile id in use, out[8] = 1 if checkpoints are held
 * per launch group, out[9] = 1 for the fused 2D schedule, out[10] / out[11] =
 * tile id of the velocity phases / of the adjoint A phase (-1 = out[7]),
 * out[12] = segments per launch group held by the replay cache, out[13] =
 * pass graphs currently instantiated.
 * HOST long long [nout]; the first min(nout, 14) entries are written.
 * Errors: EINVAL (NULL ctx or out). */
lsrtm_status lsrtm_sizes(lsrtm_ctx* ctx, long long* out, int nout);

/* Timing statistics of the last pass (HOST double [nout]); see
 * LSRTM_STAT_* for the layout.  Per-kernel times need LSRTM_OPT_TIMING.
 * Errors: EINVAL (NULL ctx or out). */
enum {
    LSRTM_STAT_PASS_MS = 0,       /* wall time of the last pass (HIP events)        */
    LSRTM_STAT_KERNEL_MS = 1,     /* [1 + 2*k], [2 + 2*k]: total ms and launch count */
    LSRTM_NKERNEL = 8             /* kernel classes: 0 born_v, 1 born_p, 2 bg_v,
                                     3 bg_p, 4 adj_a, 5 adj_b, 6 ckpt, 7 rec     */
};
lsrtm_status lsrtm_stats(lsrtm_ctx* ctx, double* out, int nout);

/* Tile shape of a tile id: out[0] = BZ, out[1] = BX.  Returns LSRTM_EINVAL
 * for an unknown id.  HOST int [2].  In 3D an id also fixes the threads per
 * block and the planes a tile marches through (results are the same bits
 * for every id):
 *   0: 64 x 4 (256 threads, 32 planes)   1: 64 x 8 (256, 32)
 *   2: 64 x 8 (256, 64)                  3: 32 x 8 (256, 64)
 *   4: 128 x 4 (256, 64)                 5: 64 x 4 (256, 64)
 *   6: 256 x 4 (1024, 32)                7: 256 x 8 (1024, 32)
 *   8: 128 x 8 (1024, 32)                9: 64 x 8 (512, 32)
 *   10: 128 x 4 (512, 32)
 * (a tile of 256 rows spans the whole padded z extent of grids up to 256
 * nodes deep; deeper grids stack such tiles with a z-halo between them). */
lsrtm_status lsrtm_tile_shape(int ndim, int tile_id, int* out);

/* Wait for the context's stream and release every device resource of the
 * context; NULL is ignored. */
void lsrtm_destroy(lsrtm_ctx* ctx);

/* Static description of a status code ("unknown status" for other values). */
const char* lsrtm_strerror(int status);

/* Description of the last error on this context ("" if none). */
const char* lsrtm_last_error(lsrtm_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* LSRTM_H */
