/*
 * scpic.h -- C ABI of libscpic, a gfx950 (MI355X) library for the per-step 2D
 * particle-in-cell space-charge loop of a proton ring (arXiv:2010.11540):
 *
 *   push    particles through the ring's elements: linear maps and thin
 *           sextupoles; with (sigma, p_sigma) also the chromatic thick
 *           quadrupole and the split thick sextupole           (Sec. III)
 *   deposit charge on a transverse grid of nodes              (Sec. IV-A)
 *   solve   the 2D Poisson equation for E                     (Sec. IV, eq. poisson3D):
 *           open boundary by Hockney's free-space Green's-function method
 *           (cited in Sec. I), or the grounded rectangular pipe (Sec. IV-B)
 *   kick    interpolate E to the particles, kick the momenta  (Sec. IV, transverse kick):
 *           cloud-in-cell or the B-spline surface of Sec. IV-C; optionally
 *           with the long-bunch line density and longitudinal kick
 *
 * Conventions
 *   - Every pointer named "device" is HIP device memory owned by the caller;
 *     the library never frees it.  Pointers named "host" are read during the
 *     call only.
 *   - Every call is asynchronous on the context's stream (see scpic_create /
 *     scpic_set_stream): it returns after enqueuing work, and results are valid
 *     once that stream has been synchronised.
 *   - Invalid arguments return SCPIC_EINVAL before any memory is touched and
 *     before anything is enqueued.  No C++ exception crosses the ABI.  The
 *     message of the last error of the calling thread is scpic_last_error().
 *   - A context serves one host thread at a time.
 *
 * Units and normalisation
 *   Particles carry (x, px, y, py): positions in m, px, py the transverse
 *   momenta normalised to the reference momentum (rad); optionally the
 *   longitudinal pair (sigma = s - c beta0 t in m, p_sigma).  Charge is counted in
 *   fixed-point units of 2^-24 of one macro-particle.  The potential solves
 *   lap(phi) = -2 pi rho with the free-space Green's function G = -ln(r), so
 *   a unit line charge has E_r = 1/r; a space-charge kick is p += kappa * E,
 *   where kappa carries the perveance, the 1/gamma^3 factor of the paper's
 *   long-bunch approximation (Sec. IV, eq. pot2) and the distance since the
 *   previous kick (Sec. IV, transverse kick).
 */
#ifndef SCPIC_H
#define SCPIC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
typedef int32_t scpic_status;
#define SCPIC_OK 0
#define SCPIC_EINVAL (-1)      /* invalid argument; nothing touched */
#define SCPIC_ENOMEM (-2)      /* device allocation failed (only in the calls
                                  documented to allocate) */
#define SCPIC_EHIP (-3)        /* a HIP runtime call failed */
#define SCPIC_EUNSUPPORTED (-4) /* valid but unsupported shape (e.g. grid size) */

/* ---- precision forms --------------------------------------------------- */
/* SCPIC_FP64:  every step in FP64 (fields are double arrays).
 * SCPIC_MIXED: coordinates, maps and kick accumulation FP64; the charge grid
 *              is exact fixed point as in FP64; the Poisson solve, the field
 *              and its interpolation are FP32 (fields are float arrays). */
#define SCPIC_FP64 0
#define SCPIC_MIXED 1

/* ---- grid -------------------------------------------------------------- */
/* nx x ny nodes at (x_min + i dx, y_min + j dy); node arrays are row-major,
 * index i*ny + j (i along x).  A particle belongs to the domain when
 * 0 <= (x - x_min) * (1/dx) < nx - 1 and likewise in y (each product and the
 * reciprocal evaluated in FP64, correctly rounded); a NaN coordinate does not.
 * Supported: nx in [8, 256], ny a multiple of 4 in [8, 256] (the paper's
 * 100 x 100 grid, Sec. IV-A, among them); the grounded pipe solver
 * (SCPIC_OPT_SOLVER) needs powers of two.  Other sizes: SCPIC_EUNSUPPORTED. */
typedef struct {
    int32_t nx, ny;
    double x_min, y_min, dx, dy;
} scpic_grid;

/* ---- particles --------------------------------------------------------- */
/* Structure of arrays, n entries each, device, contiguous FP64.
 * w (device, n floats, may be NULL): per-particle kick weight w_p; a kick
 * adds kappa * w_p * E (w_p = 1 when NULL).  This is the 2.5D long-bunch
 * form of Sec. IV (eq. poisson3D, eq. pot2): the transverse field of the
 * whole beam's transverse distribution, scaled by the line density
 * lambda(z_p) at the particle (w_p = lambda(z_p) / lambda_peak).  The deposit
 * is unweighted.
 * lost (device, n bytes, may be NULL): nonzero marks a particle that has left
 * the grid domain at a deposit or kick; a lost particle is frozen (no push,
 * kick or deposit) and keeps its last coordinates.  With lost == NULL,
 * particles outside the domain simply take no part in deposit and kick.
 * sigma, psigma (device, n doubles each, may both be NULL): the longitudinal
 * canonical pair of Sec. III, sigma = s - c beta0 t (m) and p_sigma.  Required
 * (SCPIC_EINVAL otherwise) when a lattice holds thick elements, which advance
 * sigma and read p_sigma; every other element leaves both alone. */
typedef struct {
    double *x, *px, *y, *py;
    const float *w;
    uint8_t *lost;
    int64_t n;
    double *sigma, *psigma;
} scpic_particles;

/* ---- lattice elements (Sec. III) --------------------------------------- */
/* kind:
 *   SCPIC_EL_LIN2X2     p[0..3] x-plane matrix on (x, px), p[4..7] y-plane
 *                       matrix on (y, py), both row-major: v <- M v
 *   SCPIC_EL_LIN4X4     p[0..15] row-major matrix on (x, px, y, py)
 *   SCPIC_EL_SEXT_THIN  p[0] = k2*L: the kick step of the split thick
 *                       sextupole (Sec. III-C) with V = k2 (x^3 - 3 x y^2)/6:
 *                       px -= (k2L/2)(x^2 - y^2),  py += k2L x y
 *   SCPIC_EL_SC         p[0] = kappa: a space-charge location (deposit,
 *                       solve and kick with coefficient kappa)
 *   SCPIC_EL_QUAD_THICK p[0] = k1 (1/m^2, > 0 focuses x), p[1] = L (m),
 *                       p[2] = 1/gamma0^2: the thick quadrupole with
 *                       chromatic focusing of Sec. III-B, the exact flow of
 *                       H_approx (eq. H) over L; with q = 1 - p_sigma each
 *                       plane turns by sqrt(|k1| q) L (cos/sin in the
 *                       focusing plane, cosh/sinh in the other) and
 *                       sigma += p_sigma L/gamma0^2 - (1/2) int (px^2+py^2) ds
 *   SCPIC_EL_SEXT_THICK p[0] = k2 (1/m^3), p[1] = L (m), p[2] = 1/gamma0^2,
 *                       p[3] = n (an integer in [1, 1024]): the thick
 *                       sextupole of Sec. III-C, n times the symmetric product
 *                       of exact flows H0 (a h), V (h/2), H0 (c h), V (h/2),
 *                       H0 (a h) with h = L/n, c = 1/sqrt 3, a = (1 - c)/2,
 *                       H0 = (px^2 + py^2)(1 - p_sigma)/2 + p_sigma^2/(2 gamma0^2),
 *                       V = k2 (x^3 - 3 x y^2)/6; k2 = 0 is the exact drift
 *                       (p[4..15] are ignored; a drift next to a thick
 *                       sextupole of the same gamma0 may be folded into its
 *                       first or last H0 flow, which the exact flows allow)
 * The thick elements need the particles' sigma and psigma and are evaluated in
 * FP64: the on-momentum angles' sin, cos, sinh and cosh and the sextupole's
 * step lengths once per element on the host, each particle's chromatic
 * correction by series and angle doubling and its sqrt(1 - p_sigma) on the
 * device (results agree with any other correctly implemented evaluation to
 * rounding, not bit for bit).
 * Linear maps are evaluated as written in row order, left to right, with no
 * fused multiply-add, so a push is bit-identical to the same sums in IEEE
 * FP64.  sizeof(scpic_element) == 136. */
#define SCPIC_EL_LIN2X2 1
#define SCPIC_EL_LIN4X4 2
#define SCPIC_EL_SEXT_THIN 3
#define SCPIC_EL_SC 4
#define SCPIC_EL_QUAD_THICK 5
#define SCPIC_EL_SEXT_THICK 6
typedef struct {
    int32_t kind;
    int32_t reserved;
    double p[16];
} scpic_element;

typedef struct scpic_ctx scpic_ctx;

/* Beam diagnostics over the particles not lost:
 *   alive    particles with lost == 0 (all of them without a lost array);
 *   mean     <x>, <px>, <y>, <py> over them;
 *   emit_x   sqrt(<dx^2><dpx^2> - <dx dpx>^2), d the deviation from the mean
 *            (population moments, FP64); emit_y likewise in (y, py).
 * With no particle alive every field is 0. */
typedef struct {
    int64_t alive;
    double mean[4];
    double emit_x, emit_y;
} scpic_diag;

/* Library version as 10000*major + 100*minor + patch. */
int32_t scpic_version(void);

/* Message of the calling thread's last error ("" if none).  The pointer stays
 * valid until the thread's next scpic call. */
const char *scpic_last_error(void);

/* Create a context for one grid geometry and precision form on the current
 * HIP device: the cells and representative grid points of the particle-in-cell
 * cycle (Sec. I), here the transverse node grid of the charge density and the
 * Poisson solve (Sec. IV, Sec. IV-A: the grid sized so that one copy of the
 * charge grid sits in on-chip memory).  It allocates every workspace (per-block charge partials, FFT
 * spectra, the Green's-function spectrum and the internal field); afterwards
 * only scpic_set_line_density and SCPIC_OPT_GATHER's first use allocate device
 * memory (their own buffers), never a push, deposit, solve, kick or track.  hip_stream: the hipStream_t to enqueue
 * on (NULL = the null stream).  The Green's-function spectrum is computed
 * here, once. */
scpic_status scpic_create(scpic_ctx **out, const scpic_grid *grid, int32_t precision,
                          void *hip_stream);

/* Free a context's workspaces (synchronises its stream first).  NULL is a no-op. */
scpic_status scpic_destroy(scpic_ctx *ctx);

/* Change the stream later calls enqueue on. */
scpic_status scpic_set_stream(scpic_ctx *ctx, void *hip_stream);

/* Push the particles through elements[0..n_el) in order (host array).
 * SCPIC_EL_SC entries are skipped.  Lost particles are not moved. */
scpic_status scpic_push(scpic_ctx *ctx, const scpic_particles *parts,
                        const scpic_element *elements, int32_t n_el);

/* Cloud-in-cell charge deposit (Sec. IV-A).  Each particle in the domain adds
 * to the four nodes of its cell the integer weights
 *   (4096-a)(4096-b), a(4096-b), (4096-a)b, ab   at (i,j), (i+1,j), (i,j+1), (i+1,j+1),
 * with t = (x - x_min)*(1/dx), i = floor(t), a = floor((t-i)*4096 + 0.5) (all
 * FP64) and likewise b in y: the paper's bilinear fractions rounded to 12 bits
 * per axis, summing to exactly 2^24 per particle.
 * rho (device, nx*ny int64) is overwritten with the exact integer sums; the
 * result does not depend on particle order or launch shape.  Particles outside
 * the domain are marked lost.  n_in (device, one int64, may be NULL) receives
 * the number of particles deposited. */
scpic_status scpic_deposit(scpic_ctx *ctx, const scpic_particles *parts, int64_t *rho,
                           int64_t *n_in);

/* Open-boundary field of a charge grid: the potential is the linear
 * convolution of rho*scale with G(X,Y) = -ln(X^2+Y^2)/2 over node offsets
 * (G(0,0) = the average of G over one cell), taken by a zero-padded
 * mx x my FFT convolution (mx, my the smallest powers of two >= 2nx, 2ny);
 * the field is the centred difference
 *   ex = -(phi[i+1][j] - phi[i-1][j]) / (2 dx),  ey likewise,
 * at the nodes 0..nx-1 x 0..ny-1 (both evaluated spectrally).
 * rho: device, nx*ny int64.  ex, ey: device, nx*ny, double (SCPIC_FP64) or
 * float (SCPIC_MIXED), row-major. */
scpic_status scpic_solve(scpic_ctx *ctx, const int64_t *rho, double scale, void *ex, void *ey);

/* Interpolate the node field to each particle with the same four weights as
 * the deposit (divided by 2^24) and kick: px += kappa*Ex, py += kappa*Ey.
 * ex, ey: device, as produced by scpic_solve for this context.  Lost particles
 * are skipped; particles outside the domain are marked lost. */
scpic_status scpic_kick(scpic_ctx *ctx, const scpic_particles *parts, const void *ex,
                        const void *ey, double kappa);

/* Track n_turns through the one-turn sequence turn[0..n_el) (host array).
 * This is the particle-in-cell cycle of Sec. I repeated over the ring's
 * components and turns: charge assignment, Poisson solve, then motion in
 * the solved field, with the single-particle maps of Sec. III between the
 * space-charge locations and the space-charge kick of Sec. IV (its length L
 * the distance since the previous location, carried by kappa).
 * Non-SC elements are pushed in order; at each SCPIC_EL_SC element the beam's
 * charge is deposited, the field solved with scale 1/(2^24 * parts->n) (the
 * charge of lost particles leaves with them) and every particle kicked with
 * that element's kappa.  Equivalent to the sequence of scpic_push /
 * scpic_deposit / scpic_solve / scpic_kick calls (with the line density or
 * the B-spline gather on, to the steps those options describe), fused: each kick, the
 * following push and the next deposit run as one pass over the particles, and
 * one turn runs as one captured HIP graph.  Turn graphs are cached per
 * (particle arrays, lattice); at most 8 are kept. */
scpic_status scpic_track(scpic_ctx *ctx, const scpic_particles *parts, const scpic_element *turn,
                         int32_t n_el, int32_t n_turns, scpic_diag *diag);

/* Diagnostics of parts as they stand (after the work already queued on the
 * context's stream): two passes over the particles on the device (the sums,
 * then the centred second moments), each reduced in a fixed order, so the
 * result does not depend on scheduling.  out: host; the call waits for the
 * stream.  scpic_track fills its diag argument (host, may be NULL) the same
 * way after the last turn, and then waits too.  Not for stream capture.
 * The emittance is the usual rms definition, not an equation of the paper.
 * Errors: SCPIC_EINVAL for a NULL context, particle set or out (checked
 * before any device work); SCPIC_EHIP if a launch or the copy fails. */
scpic_status scpic_diagnose(scpic_ctx *ctx, const scpic_particles *parts, scpic_diag *out);

/* Options (scpic_set_option):
 *   SCPIC_OPT_USE_GRAPH      1 (default): scpic_track replays one HIP graph
 *                            per turn; 0: it launches the same kernels directly.
 *   SCPIC_OPT_PASS_BLOCKS    workgroups of the particle pass (0 = automatic:
 *                            one per compute unit).
 *   SCPIC_OPT_PASS_THREADS   threads per workgroup of the particle pass
 *                            (256, 512 or 1024; default 1024).
 *   SCPIC_OPT_SOLVER         SCPIC_SOLVER_OPEN (default): the open-boundary
 *                            convolution of scpic_solve's comment;
 *                            SCPIC_SOLVER_PIPE (nx and ny powers of two, else
 *                            SCPIC_EUNSUPPORTED): the grounded rectangular pipe
 *                            of Sec. IV-B -- the 5-point discrete Poisson
 *                            equation lap phi = -2 pi rho / (dx dy) with
 *                            phi = 0 on walls through node 0 and node nx along
 *                            x (node nx is one spacing past the last node),
 *                            and node 0 and node ny along y; the charge on the
 *                            wall nodes i = 0 or j = 0 goes to the wall.
 *                            Solved by the paper's odd extension and DFT,
 *                            each mode divided by the Laplacian's eigenvalue.
 *                            Applies to scpic_solve, scpic_track and
 *                            scpic_reduce_solve; waits for the context's
 *                            stream and drops its cached turn graphs.
 *   SCPIC_OPT_GATHER         SCPIC_GATHER_CIC (default): the kick gathers the
 *                            node field with the deposit's four weights;
 *                            SCPIC_GATHER_BSPLINE: the interpolation of
 *                            Sec. IV-C, read as the uniform bicubic B-spline
 *                            with the node potentials as control points --
 *                            phi(x, y) = sum_{m,n=0..3} u[i+m-1][j+n-1]
 *                            B_m(tx) B_n(ty) over the 4x4 nodes around the
 *                            particle's cell (tx, ty its exact cell
 *                            fractions, B the uniform cubic basis) -- and the
 *                            kick takes E = -grad phi analytically.  The
 *                            solve then also keeps the potential on nodes
 *                            -1..nx by -1..ny (scpic_get_potential).  Applies
 *                            to scpic_track and scpic_pass (scpic_kick gathers
 *                            the field it is given); not with the line
 *                            density.  Allocates the potential's buffers on
 *                            first use, waits for the stream and drops the
 *                            cached turn graphs.
 * Results do not depend on the launch shape. */
#define SCPIC_OPT_USE_GRAPH 1
#define SCPIC_OPT_PASS_BLOCKS 2
#define SCPIC_OPT_PASS_THREADS 3
#define SCPIC_OPT_SOLVER 4
#define SCPIC_SOLVER_OPEN 0
#define SCPIC_SOLVER_PIPE 1
#define SCPIC_OPT_GATHER 5
#define SCPIC_GATHER_CIC 0
#define SCPIC_GATHER_BSPLINE 1
scpic_status scpic_set_option(scpic_ctx *ctx, int32_t option, int64_t value);

/* Fused particle pass, one launch: optionally kick with the context's
 * internal field (kappa; skipped when kick == 0), push through
 * elements[0..n_el) (at most 12, no SC entries), then optionally deposit into
 * the context's per-block charge partials (deposit != 0).  This is one step
 * of scpic_track exposed for timing; scpic_pass followed by scpic_reduce_solve
 * completes the step. */
scpic_status scpic_pass(scpic_ctx *ctx, const scpic_particles *parts, int32_t kick, double kappa,
                        const scpic_element *elements, int32_t n_el, int32_t deposit);

/* Grid phase of one step: sum the per-block partials of the last depositing
 * scpic_pass, solve with the given scale into the context's internal field. */
scpic_status scpic_reduce_solve(scpic_ctx *ctx, double scale);

/* Copy the context's internal field (written by scpic_track /
 * scpic_reduce_solve) to ex, ey (device; double or float per precision). */
scpic_status scpic_get_field(scpic_ctx *ctx, void *ex, void *ey);

/* Long-bunch line density (Sec. IV).  nz > 0 turns it on for scpic_track and
 * scpic_pass / scpic_reduce_solve (the per-element calls scpic_deposit,
 * scpic_solve and scpic_kick stay transverse); nz = 0 turns it off.  At every
 * space-charge step the line density lambda(sigma) is histogrammed on the nz
 * nodes z_min + k dz with the one-dimensional form of the charge assignment
 * (t = (sigma - z_min)(1/dz), k = floor(t), a = floor((t - k) 4096 + 0.5),
 * weights 4096 - a at k and a at k + 1, exact integer sums), together with the
 * transverse charge; the node tables are
 *   lw[k] = h[k] / max h,   ld[k] = (h[k+1] - h[k-1]) / (2 dz max h)
 * (h = 0 beyond the line).  Each kick then, with w and d interpolated from lw
 * and ld with the particle's line weights and phi, E with its transverse
 * weights, applies
 *   px += kappa w Ex,  py += kappa w Ey,  p_sigma -= gamma0 kappa phi d:
 * the transverse kick scaled by lambda(sigma)/lambda_peak and the longitudinal
 * kick of Sec. IV, whose coefficient e/(m gamma0^2 beta0^2 c^2) is gamma0 times
 * the transverse one (carried by kappa).  phi is the potential of the grounded
 * pipe: the line density needs SCPIC_SOLVER_PIPE (SCPIC_EUNSUPPORTED at track
 * time otherwise), the particles' sigma and psigma, and no per-particle
 * weights w (SCPIC_EINVAL), and the cloud-in-cell gather (SCPIC_EUNSUPPORTED
 * with SCPIC_GATHER_BSPLINE).  A particle whose sigma leaves [z_min,
 * z_min + (nz-1) dz) is lost like one leaving the grid.
 * nz in [8, 512], dz > 0, gamma0 >= 1, all finite.  This call synchronises the
 * context's stream and allocates the line's buffers (the histograms of up to
 * the context's largest workgroup count and the node tables; the node
 * potential and its spectrum once); tracking allocates nothing. */
scpic_status scpic_set_line_density(scpic_ctx *ctx, int32_t nz, double z_min, double dz,
                                    double gamma0);

/* Copy the line tables of the last solve, lw and ld (device, nz doubles
 * each; either may be NULL).  SCPIC_EINVAL when the line density is off. */
scpic_status scpic_get_line_state(scpic_ctx *ctx, double *lw, double *ld);

/* Copy the node potential of the last solve (device, (nx+2)*(ny+2) doubles or
 * floats per precision, row-major: node (i, j) for i = -1..nx, j = -1..ny at
 * [(i+1)*(ny+2) + j+1]), the potential whose centred differences are the
 * field.  Kept while the line density or the B-spline gather is on
 * (SCPIC_EINVAL otherwise). */
scpic_status scpic_get_potential(scpic_ctx *ctx, void *phi);

/* ---- batches of independent beams --------------------------------------
 * Many independent beams (a tune scan, Sec. V; beams of different sizes on
 * different grids) tracked together: every particle pass and every grid
 * phase is one launch over all beams, each beam keeping its own particles,
 * grid, partials, field, ring and kick strengths.  Each beam's result is the
 * one scpic_track gives for that beam alone. */
typedef struct scpic_batch scpic_batch;

/* Create a batch of n_inst beams (1 <= n_inst <= 4096).  Beam k owns the
 * particles offsets[k] .. offsets[k+1]-1 of the concatenated arrays given to
 * scpic_track_batched, and the grid grids[k] (the limits of scpic_create).
 * offsets: host, n_inst + 1 entries, offsets[0] == 0, non-decreasing.
 * grids: host, n_inst entries.  precision: as scpic_create.  hip_stream: the
 * stream every call of the batch uses (NULL = default stream).  All
 * workspaces are allocated here; beams with equal grids share the Green's
 * spectrum and twiddle tables.  Errors: SCPIC_EINVAL (NULL or inconsistent
 * arguments), SCPIC_EUNSUPPORTED (grid limits), SCPIC_ENOMEM, SCPIC_EHIP;
 * *out is NULL on error. */
scpic_status scpic_batch_create(scpic_batch **out, const scpic_grid *grids,
                                const int64_t *offsets, int32_t n_inst, int32_t precision,
                                void *hip_stream);

/* Release a batch (waits for its stream).  NULL is accepted. */
scpic_status scpic_batch_destroy(scpic_batch *b);

/* Stream for the batch's later calls (NULL = default stream). */
scpic_status scpic_batch_set_stream(scpic_batch *b, void *hip_stream);

/* Track every beam n_turns turns through its own ring, as scpic_track does
 * for one beam: the particle-in-cell cycle of Sec. I with the maps of
 * Sec. III and the kick of Sec. IV, for independent beams such as the
 * points of a tune scan (Sec. V compares tunes and their spread across
 * settings).  Same kick placement, same normalisation 1/(2^24 N0_k) with
 * N0_k = offsets[k+1] - offsets[k], same lost-particle rules).
 * parts: the concatenated beams (parts->n == offsets[n_inst]; w and lost
 * may be NULL).  turns[k]: host array of n_els[k] elements, beam k's ring.
 * The rings must share one schedule: the same number of SC elements, and in
 * each stretch between consecutive SC elements (the stretch after the last
 * SC element joined to the one before the first) at most 12 other elements;
 * otherwise SCPIC_EUNSUPPORTED.  The step tables of a schedule are cached on
 * the device (at most 16 schedules; one turn is one captured HIP graph). */
scpic_status scpic_track_batched(scpic_batch *b, const scpic_particles *parts,
                                 const scpic_element *const *turns, const int32_t *n_els,
                                 int32_t n_turns);

/* Pick the launch shape of the batched particle pass by timing it: for each
 * candidate (threads per workgroup 256, 512 or 1024; workgroups per compute
 * unit over the whole batch 1, 2 or 4, which sets the particles per
 * workgroup and the number of LDS charge-grid copies and partial slices of
 * each beam) one untimed and trial_turns timed turns run on a device scratch
 * copy of parts (allocated and freed here; parts itself is not modified),
 * and the fastest candidate is kept for later scpic_track_batched calls.
 * Results do not depend on the shape.  threads_out, blocks_per_cu_out (host,
 * may be NULL) receive the choice.  trial_turns in [1, 100].  Drops the
 * batch's cached schedules; waits for the batch's stream. */
scpic_status scpic_batch_autotune(scpic_batch *b, const scpic_particles *parts,
                                  const scpic_element *const *turns, const int32_t *n_els,
                                  int32_t trial_turns, int32_t *threads_out,
                                  int32_t *blocks_per_cu_out);

/* Copy beam k's node field after its last solve to ex, ey (device, nx*ny
 * each, double or float per precision). */
scpic_status scpic_batch_get_field(scpic_batch *b, int32_t k, void *ex, void *ey);

/* ---- deposit without allocation ----------------------------------------
 * For callers that cannot allocate device memory: code being captured into a
 * HIP graph, tight serving loops, harnesses that forbid hipMalloc.  The same
 * cloud-in-cell deposit as scpic_deposit (same weights, same exact integer
 * result, which does not depend on the launch shape) without a context: its
 * per-workgroup charge partials, their headers and the carry grid live in a
 * static device array of the library, SCPIC_STATIC_SCRATCH_BYTES per device,
 * held by every device the library runs on until the process ends.  Nothing
 * is allocated: no hipMalloc or hipFree, no memset nodes (the scratch it needs
 * cleared is cleared by a kernel at the start of each call), so the call can
 * be captured.  The first call on a device looks up the array's address on
 * that device and sets the pass kernels' LDS limit (both outside any capture
 * on that device: make one uncaptured call first).
 * grid: host, the limits of scpic_create.  parts: as scpic_deposit (lost may
 * be NULL; out-of-domain particles are marked lost when it is not).
 * rho: device, nx*ny int64, overwritten.  n_in: device, one int64, may be
 * NULL.  hip_stream: the stream to enqueue on (NULL = the null stream).
 * Every call on one device shares that device's array and leaves its own
 * contents in it: calls that overlap on one device (on different streams, or
 * from different host threads) race and must be serialised by the caller.
 * Errors, before anything is enqueued: SCPIC_EINVAL (NULL grid, particles or
 * rho; bad particle arrays or grid spacing), SCPIC_EUNSUPPORTED (grid beyond
 * scpic_create's limits, or more than 64 * (2^31 - 1) particles); SCPIC_EHIP
 * if the address lookup or a launch fails. */
#define SCPIC_STATIC_SCRATCH_BYTES 17303552 /* 64 workgroups' partials of a
                                               65536-node grid, their headers
                                               and a 65536-node carry grid */
scpic_status scpic_deposit_static(const scpic_grid *grid, const scpic_particles *parts,
                                  int64_t *rho, int64_t *n_in, void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* SCPIC_H */
