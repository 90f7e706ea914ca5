/*
 * fw25.h -- C ABI of the MI355X (gfx950) FDTD step for attenuating, nonlinear
 * acoustic waves with multiple relaxation mechanisms.
 *
 * The method (Sode & Pinton, "Spatially heterogeneous power-law attenuation
 * with multiple relaxation mechanisms for ultrasound modeling"):
 *   - Sec. 2.1, Eqs. (wave1)/(wave2): staggered pressure p and particle
 *     velocity v, rho dv/dt = -grad~ p, kappa dp/dt = -div~ v (K = 1/kappa).
 *   - Sec. 2.1, Eq. (relaxation4): every derivative is stretched,
 *     d/dx~ = (1/kappa_i) d/dx + sum_nu psi_i^nu, i = 1 (gradient) or 2
 *     (divergence), nu = 1..N relaxation mechanisms.
 *   - Sec. 2.1, Eqs. (relaxation_psi), (relaxation_a), (relaxation_b): the
 *     memory variables follow psi <- b psi + a D with
 *     b = exp(-(d/kappa + alpha) dt), a = d / (kappa (d + kappa alpha)) (b - 1).
 *   - Sec. 2.1 / abstract: the CPML boundary reuses the same recursion form.
 *   - Sec. 3.3: staggered finite differences of order 2M in space, M = 4.
 *   - Sec. 1 names pressure-dependent nonlinearity; here K -> K + 2 beta p.
 *
 * Conventions for every call:
 *   - Return value: FW_OK (0) or a negative fw_status.  No C++ exception
 *     crosses this boundary.  fw_last_error() returns a thread-local text.
 *   - Grids: cell (i, j, k) of a domain with shape (nx, ny, nz) has the
 *     domain-local linear index (k*ny + j)*nx + i (x fastest).  Unused
 *     trailing dimensions are 1.  The face i+1/2 of an axis is stored at the
 *     index of cell i.  Field values beyond the grid are zero.
 *   - Several domains ("shots", ragged sizes) can share one object; they all
 *     advance together with the same dx, dt, N and CPML width.
 *   - Memory: device state lives in a caller-owned workspace (for example a
 *     torch uint8 tensor) bound with fw_bind_workspace; the library borrows
 *     it and never frees it.  The library allocates only small device tables
 *     (class coefficients, CPML profiles, tile lists, sources, receivers,
 *     counters).  Host arrays passed to setters are copied before return.
 *   - Streams: hip_stream is a hipStream_t (NULL = default stream).  Work is
 *     enqueued asynchronously unless stated otherwise.
 *   - Call order: create -> bind_workspace -> set_media ->
 *     set_relaxation_table -> [set_sources] -> [set_receivers] -> step.
 *     A call made too early returns FW_ESTATE.
 */
#ifndef FW25_H
#define FW25_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fw_sim fw_sim;

typedef enum fw_status {
    FW_OK = 0,
    FW_EINVAL = -1,        /* bad argument (shape, index, count, pointer) */
    FW_ESTATE = -2,        /* call out of order                          */
    FW_EUNSTABLE = -3,     /* time step violates the stability bound     */
    FW_EHIP = -4,          /* HIP runtime error (text has the HIP error) */
    FW_ENOMEM = -5,        /* workspace too small / allocation failed    */
    FW_ENONFINITE = -6,    /* non-finite value detected                  */
    FW_EUNSUPPORTED = -7   /* valid request this build does not support  */
} fw_status;

/* Thread-local text of the last failure on this thread ("" if none). */
const char *fw_last_error(void);

/* ABI version, incremented on every incompatible change. */
int fw_abi_version(void);

/*
 * Create a grid object (host only, no device work).
 *   ndim       1, 2 or 3.
 *   n_domains  >= 1.
 *   shape      [n_domains][3] = (nx, ny, nz); dims beyond ndim must be 1;
 *              every used dim must exceed 2*pml_cells + 8.
 *   dx, dt     grid step (m) and time step (s), both > 0.
 *   n_mech     relaxation mechanisms N per operator, 1..4 (Sec. 2.1).
 *   pml_cells  CPML width P in cells on every face of every domain (>= 0).
 *   pml_params NULL for defaults, else [3] = (R0, f_alpha_hz, c_ref):
 *              d(delta) = d0 delta^2 with d0 = 3 c_ref ln(1/R0) / (2 P dx),
 *              alpha(delta) = pi f_alpha (1 - delta), kappa = 1, delta the
 *              depth into the slab measured from its inner edge at positions
 *              P - 1/2 and n - P - 1/2 (defaults 1e-4, 1e6, 0; c_ref = 0 takes
 *              the largest class speed given to fw_set_media).  Inside the
 *              slab of an axis the CPML recursion acts on that axis'
 *              derivative before the tissue recursions do, so the layer's
 *              stretch is the product of the CPML and tissue stretches (the
 *              layer stretches the coordinate of the lossy medium; the tissue
 *              mechanisms continue inside it).
 * On success *out holds a new object owned by the caller (fw_destroy).
 */
int fw_create_grid(fw_sim **out, int ndim, int n_domains, const int64_t *shape,
                   double dx, double dt, int n_mech, int pml_cells, const double *pml_params);

/* Infrastructure (no operation of the method).  Release the object and the
 * small tables the library allocated.  The bound workspace is not freed. */
int fw_destroy(fw_sim *sim);

/* The state of Sec. 3.3's scheme: device bytes the workspace must provide:
 * pressure, velocity, the memory variables of Eq. (relaxation_psi) (3N face
 * variables and N cell variables summed over axes per cell), CPML memory
 * variables (the same recursion form, Sec. 2.1) and the uint8 class map.
 * -1 on a NULL sim. */
int64_t fw_workspace_bytes(const fw_sim *sim);

/* Infrastructure (no operation of the method).
 * Bind a caller-owned device buffer of at least fw_workspace_bytes bytes,
 * 256-byte aligned.  The state is zeroed (synchronously on the default
 * stream) and the step counter reset. */
int fw_bind_workspace(fw_sim *sim, void *d_ptr, int64_t bytes);

/*
 * Tissue classes and their map (Sec. 2.1: material maps rho(x), kappa(x)).
 *   h_class     host uint8, all domains concatenated in domain order, each in
 *               its own linear order; value = class index local to its domain.
 *   class_base  host [n_domains]: global class = class_base[d] + local index;
 *               every local index must be < 256 and the global < n_classes.
 *   c, rho      host [n_classes] sound speed (m/s) and density (kg/m^3), > 0.
 *   beta        host [n_classes] nonlinearity coefficient (K -> K + 2 beta p);
 *               0 is the linear medium, a tissue with parameter B/A has
 *               beta = 1 + B/(2A).
 *   c_noise_amp per-voxel speed perturbation c (1 + eps), eps = amp (2u - 1),
 *               u = (SplitMix64(noise_seed ^ local_index) >> 40) * 2^-24;
 *               0 disables it.  0 <= amp < 0.5.
 * Checks the stability bound c_max (1 + amp) dt/dx sqrt(ndim) sum|c_m| < 1
 * (FW_EUNSTABLE).  Uploads the map into the workspace (synchronous).
 */
int fw_set_media(fw_sim *sim, const uint8_t *h_class, const int32_t *class_base, int n_classes,
                 const double *c, const double *rho, const double *beta,
                 double c_noise_amp, uint64_t noise_seed);

/*
 * Per-voxel attenuation within a class (Sec. 1 and Sec. 4.5: attenuation
 * that varies from voxel to voxel; the paper assigns relaxation parameters
 * per pixel).  d_scale is a caller-owned device float array over all cells
 * (unpadded layout: domains concatenated, each in its own linear order),
 * borrowed until replaced or cleared (NULL), with values s(x) in [0, 1]:
 * the memory-variable coefficients a of both operators of the cell become
 * s(x) a (the relaxation times, i.e. b, stay those of the class), so the
 * relaxation strength of the class is scaled down voxel by voxel; for
 * relaxation strengths small against the medium's stiffness the attenuation
 * scales the same way, alpha(x, f) ~ s(x) alpha_class(f).  The class table
 * thus describes the most attenuating voxels of the class, and s = 1
 * reproduces it bit for bit.  The values are checked on the device
 * (FW_EINVAL if any is not a finite number in [0, 1]; synchronises the
 * stream).  The strength map adds 4 bytes per cell to each update's reads.
 * The adjoint calls return FW_EUNSUPPORTED while a map is set.
 * Requires fw_set_media.
 */
int fw_set_strength_map(fw_sim *sim, const float *d_scale, void *hip_stream);

/*
 * Staggered first-derivative coefficients c_1..c_4 of every update (Sec. 3.3:
 * an operator of order 2M in space, M = 4, with fourth order in time).  The
 * default is the Taylor set (1225/1024, -245/3072, 49/5120, -5/7168), with
 * which the leapfrog step is of second order in time.  c_ref > 0 selects the
 * time-space-domain set for the Courant number r = c_ref dt / dx: the c_m
 * solving sum_m c_m (2m - 1)^(2k - 1) = r^(2k - 2), k = 1..4 (Liu and Sen
 * 2011), which makes the 1D step of order 8 in both time and space for waves
 * at speed c_ref (the relation sin(w dt / 2) = r sum_m c_m sin((2m - 1) k dx
 * / 2) then agrees with w = c_ref k through (k dx)^7).  Along each axis of a
 * 2D or 3D grid the same holds; oblique directions keep a second-order time
 * error, since that needs the off-axis stencil points of Tan and Huang (2014),
 * which this operator does not have.  c_ref = 0 restores the Taylor set.
 * FW_EINVAL if c_ref < 0, not finite or r >= 1; FW_EUNSTABLE (the previous
 * set kept) if media are set and the stability bound of the new set fails.
 * May come before or after fw_set_media; drops a captured step graph.  The
 * adjoint uses the same coefficients, so it stays the exact transpose.
 */
int fw_set_time_space_stencil(fw_sim *sim, double c_ref);

/*
 * Widened staggered stencil for fourth order in time in every direction of a
 * 2D grid (Sec. 3.3; the off-axis construction of Tan and Huang 2014).  Each
 * axis's difference gains b times the two-point differences along that axis
 * in the two rows (columns) one cell away on the other axis; with
 * r = c_ref dt / dx, b = r^2 / 24 and the on-axis c_m solving
 * sum_m c_m (2m - 1)^(2k - 1) = r^(2k - 2) - 2 b, k = 1..4, the leapfrog
 * relation sin^2(w dt / 2) = r^2 (A_x^2 + A_y^2) matches w = c_ref |k|
 * through fourth order in k dx for every direction (the mixed terms
 * included), and through eighth order along the axes.  The divergence takes
 * the same widened stencil, so it stays the negative transpose of the
 * gradient.  c_ref = 0 restores the Taylor set (b = 0).  Only the 2D tile
 * kernels implement it: fw_step returns FW_EUNSUPPORTED on other 2D paths
 * (FW_OPT_PLANE_KERNELS 0, a persistent grid), and so does the adjoint.
 * FW_EUNSUPPORTED unless ndim = 2; otherwise the errors of
 * fw_set_time_space_stencil.  Drops a captured step graph.
 */
int fw_set_widened_stencil(fw_sim *sim, double c_ref);

/* The coefficients in use into coef5[5]: c_1..c_4 and the off-axis weight b
 * (0 unless fw_set_widened_stencil set it); dimensionless, FP64. */
int fw_get_stencil(const fw_sim *sim, double *coef5);

/*
 * Relaxation parameters per class (Sec. 2.1, Table 2 variables), FP64 in:
 *   kappa [n_classes][2], d [n_classes][2][N], alpha [n_classes][2][N]
 *   (index 0: gradient operator nabla_1, index 1: divergence nabla_2).
 * Requires kappa > 0, d >= 0, alpha >= 0, d + kappa alpha > 0.  The per-step
 * coefficients a, b of Eqs. (relaxation_a)/(relaxation_b) are computed in
 * FP64 on the host and rounded to FP32 for the device.  Re-checks the
 * stability bound with 1/sqrt(min kappa_1 kappa_2).
 * The parameters are used as given.  The recursion keeps each mechanism's
 * DC gain but realises the rate r = d/kappa + alpha as (e^{r dt} - 1)/dt, so
 * a fit of the continuous model reaches its attenuation only where
 * r dt << 1; mechanisms fitted without regard to dt should be mapped to the
 * time step first (same kappa and DC gains, rate ln(1 + r dt)/dt).
 */
int fw_set_relaxation_table(fw_sim *sim, int n_classes, const double *kappa,
                            const double *d, const double *alpha);

/*
 * Sources (Sec. 4.1: plane-wave sources of Gaussian-modulated sinusoidal
 * pulses; Sec. 4.5: transducer elements; the paper does not state how a
 * source enters the scheme, the reading here is an additive soft source).
 * Additive pressure sources: after the pressure update of step t (0-based,
 * counted from the last reset), p[domain[s], cell[s]] += waves[wave_idx[s]][t]
 * for t < n_t.  cell = domain-local linear index.  Each (domain, cell) pair
 * may appear once.  waves is host float [n_wave][n_t].  n_src = 0 clears.
 */
int fw_set_sources(fw_sim *sim, int64_t n_src, const int32_t *domain, const int64_t *cell,
                   const int32_t *wave_idx, int n_wave, const float *waves, int n_t);

/*
 * Receivers (Sec. 4.1: receiver pixels recording the pressure wavefield,
 * Sec. 4.3 and Sec. 4.5: incident/reflected pressure and RF traces).
 * Receivers: after step t's sources, trace[t][r] = p[domain[r], cell[r]]
 * for t < n_t_max (later steps are not recorded).  Allocates the device
 * trace buffer [n_t_max][n_rec] (zeroed); fw_set_receivers_into takes a
 * caller-owned one instead.  n_rec = 0 clears.
 */
int fw_set_receivers(fw_sim *sim, int64_t n_rec, const int32_t *domain, const int64_t *cell,
                     int n_t_max);

/*
 * The same receivers (Sec. 4.1), recorded into a caller-owned device buffer
 * d_traces of `capacity` floats instead of one the library allocates: the
 * library zeroes its first n_rec * max(n_t_max, 1) floats ([n_t_max][n_rec],
 * row-major) and writes the traces there at every step; fw_read_receivers
 * and fw_reset_state use it.  The caller keeps it alive and unmodified while
 * the simulation steps (the library only borrows it), until receivers are
 * set again.  FW_EINVAL if d_traces is NULL with n_rec > 0 or capacity is
 * too small.  The small per-cell receiver tables are still the library's.
 */
int fw_set_receivers_into(fw_sim *sim, int64_t n_rec, const int32_t *domain, const int64_t *cell,
                          int n_t_max, float *d_traces, int64_t capacity);

/*
 * Set-up only (the step itself is that of fw_step, Sec. 3.3).
 * Do now the set-up work the next fw_step would do first: build the tile
 * lists if an option or the media changed them, and capture and instantiate
 * the graph of FW_OPT_GRAPH_STEPS steps if it is not current, so that the
 * following fw_step calls only launch (for callers that time steps or must
 * keep set-up out of a latency-bound loop).  Launches no kernel and leaves
 * the state unchanged.  FW_ESTATE before the workspace, media and relaxation
 * table are set; FW_EHIP if capture fails.
 */
int fw_prepare(fw_sim *sim);

/*
 * The FDTD step of Sec. 3.3 applied to Eqs. (wave1)/(wave2) of Sec. 2.1,
 * with the memory variables of Eq. (relaxation_psi) (staggered stencil of
 * order 8 in space, leapfrog in time).
 * Advance every domain by n_steps time steps on hip_stream (asynchronous).
 * One step = velocity update (gradient, N memory variables per axis, CPML)
 * -> pressure update (divergence, N memory variables, CPML, nonlinearity)
 * -> sources -> receivers (with the finite check of fw_first_nonfinite_step)
 * -> device step counter + 1.  Replays captured HIP graphs of the configured
 * length, with eager launches for the remainder.
 */
int fw_step(fw_sim *sim, int n_steps, void *hip_stream);

/*
 * The simulation's output, the receiver pressure traces (Sec. 4.1, Sec. 4.5).
 * Copy n_elems floats of the trace buffer ([n_t_max][n_rec], row-major) to
 * dst (device memory if dst_is_device, else host).  Synchronises the stream.
 */
int fw_read_receivers(fw_sim *sim, float *dst, int64_t n_elems, int dst_is_device, void *hip_stream);

/* The zero initial state of the time iteration (Sec. 3.3; the fields start
 * at rest before the source of Sec. 4.1 acts).  Zero every state field, the
 * traces and the step counter, and clear the finite-check flag
 * (asynchronous). */
int fw_reset_state(fw_sim *sim, void *hip_stream);

/* Infrastructure: host view of the number of time steps (Sec. 3.3) enqueued
 * since the last reset. */
int fw_get_step(const fw_sim *sim, int64_t *step);

/*
 * Instability monitor (Sec. 4.6 and Sec. 5.5 watch the recorded wavefield
 * for NaN or Inf at every step to detect divergence).
 * Finite check of every step: the source/receiver kernel (part of every
 * step, inside captured graphs too, no extra launch) flags the first trace
 * row, i.e. the 0-based step index as in fw_read_receivers, that holds a
 * NaN or infinite receiver value.  *row receives that row, or -1 if none
 * since the last reset (only rows below n_t_max are recorded and checked).
 * Synchronises the stream.  fw_energy_step checks the whole field instead.
 */
int fw_first_nonfinite_step(fw_sim *sim, int64_t *row, void *hip_stream);

/* Infrastructure (checkpoints of the time iteration of Sec. 3.3).
 * Bytes of a full state snapshot (fields, memory variables, CPML variables,
 * the step counter and the first non-finite trace row of
 * fw_first_nonfinite_step); -1 on a NULL sim. */
int64_t fw_state_bytes(const fw_sim *sim);

/* Infrastructure (checkpoints of the time iteration of Sec. 3.3).
 * Copy the full state into / out of a caller-owned device buffer of
 * fw_state_bytes bytes (asynchronous, device-to-device).  Resuming from a
 * saved state reproduces the uninterrupted run bit for bit; loading a state
 * also restores the non-finite row it was saved with, so a row flagged after
 * the save is forgotten. */
int fw_save_state(fw_sim *sim, void *d_dst, void *hip_stream);
int fw_load_state(fw_sim *sim, const void *d_src, void *hip_stream);

/*
 * Power-law attenuation coefficient alpha0 of each class (Sec. 3.1, the
 * alpha0 of alpha(f) = alpha0 f^y that the class's relaxation table was
 * fitted to), host double [n_classes], every value finite and > 0
 * (FW_EINVAL otherwise: a class without attenuation has no relaxation
 * strength to scale).  Used only by fw_adjoint's dJ/dalpha0, whose units
 * are those of J per unit of the alpha0 given here.  Requires fw_set_media.
 */
int fw_set_class_alpha0(fw_sim *sim, int n_classes, const double *alpha0);

/*
 * Discrete adjoint with checkpointed recomputation (linear media: beta = 0).
 * The paper has no adjoint; this differentiates the scheme of Sec. 2.1 and
 * Sec. 3.3 (the transposed velocity and pressure updates, memory-variable
 * and CPML recursions included, applied to every step in reverse order).
 *
 * Misfit J is any function of the receiver traces; the caller supplies
 * d_adj_src[t][r] = dJ/d trace[t][r] (device float [n_steps][n_rec]).
 * Gradients are accumulated (+=) per cell in the caller's unpadded cell
 * layout (domains concatenated, each in its own linear order):
 *   d_grad_c[x]      = dJ/dc(x) of the cell's sound speed, with the cell's
 *                      modulus K = rho c^2 (1 + eps)^2 (eps the speed
 *                      perturbation of fw_set_media), i.e. 2 rho c (1 + eps)^2
 *                      dJ/dK(x);
 *   d_grad_alpha0[x] = dJ/dalpha0(x) when the relaxation strengths d of the
 *                      cell scale with its alpha0 (kappa and alpha fixed:
 *                      d(x) = d_class alpha0(x) / alpha0_class), i.e.
 *                      dJ/ds(x) / alpha0_class for the scale s of every d of
 *                      the cell.  May be NULL; otherwise fw_set_class_alpha0
 *                      must have been called (FW_ESTATE).
 * The chain rule runs on the device (the speed perturbation is evaluated as
 * in the forward step); rho, c and alpha0 are those of the cell's class.
 *
 * d_work is a caller-owned, 256-byte aligned device buffer of
 * fw_adjoint_workspace_bytes bytes (FW_EINVAL if misaligned, FW_ENOMEM if
 * smaller) holding ceil(n_steps / ckpt_every) state checkpoints,
 * ckpt_every + 1 recomputed states, the adjoint state and scratch.
 * d_grad_c, d_grad_alpha0 and d_adj_src must be 4-byte aligned device
 * buffers of the sizes above; the gradients are accumulated into (the caller
 * zeroes them).
 * fw_forward_checkpointed resets the state, runs n_steps (recording the
 * traces) and stores the checkpoints; fw_adjoint then sweeps the segments
 * last to first, recomputing each segment's states from its checkpoint into
 * d_work.  fw_adjoint leaves the simulation's own state and step counter as
 * they were (the recompute rewrites the traces of steps < n_steps with the
 * same values), so stepping can continue after it.  fw_adjoint synchronises
 * the stream before it returns.
 * Returns FW_EUNSUPPORTED if any class has beta != 0.
 */
int64_t fw_adjoint_workspace_bytes(const fw_sim *sim, int n_steps, int ckpt_every);
int fw_forward_checkpointed(fw_sim *sim, int n_steps, int ckpt_every, void *d_work, int64_t bytes,
                            void *hip_stream);
int fw_adjoint(fw_sim *sim, int n_steps, int ckpt_every, void *d_work, int64_t bytes,
               const float *d_adj_src, float *d_grad_c, float *d_grad_alpha0, void *hip_stream);

/*
 * The same reverse sweep as fw_adjoint (the transpose of the step of
 * Sec. 3.3 applied to Eqs. (wave1)/(wave2); the paper has no adjoint: the
 * per-voxel parameters of Sec. 4.5 are what it differentiates), returning
 * the gradients before the chain rule (asynchronous): d_grad_K[x] += dJ/dK(x), the cell's bulk
 * modulus, and d_grad_s[x] += dJ/ds(x), s a scale of every relaxation
 * strength d of the cell (d -> s d, kappa and alpha fixed).  Same workspace,
 * layout and errors as fw_adjoint.
 */
int fw_adjoint_modulus(fw_sim *sim, int n_steps, int ckpt_every, void *d_work, int64_t bytes,
                       const float *d_adj_src, float *d_grad_K, float *d_grad_s, void *hip_stream);

/*
 * Measurement of the step of Sec. 3.3 (Sec. 5.3 reports the paper's run
 * times).
 * Advance n_steps steps like fw_step, but launch every kernel eagerly with a
 * HIP event before and after it on hip_stream, wait for completion, and
 * return the average time per step in milliseconds of each kernel kind:
 * avg_ms[0] velocity update, avg_ms[1] pressure update, avg_ms[2] sources and
 * receivers.  The launches are those of fw_step: with the interleaved chunk
 * schedule (FW_OPT_STEP_CHUNK) a kind's figure is the sum over its chunk
 * launches of one step.  Used for per-kernel roofline figures; the state
 * advances.
 */
int fw_time_kernels(fw_sim *sim, int n_steps, void *hip_stream, double *avg_ms);

/*
 * Diagnostics of one step (Sec. 2.1: the lossless limit of Eqs. (wave1)/
 * (wave2) conserves acoustic energy; Sec. 4.6: the peak pressure of every
 * step is watched for instability).
 * One full step (like fw_step(sim, 1, ...)) that also evaluates, per domain,
 * out[3 d + 0] = E^{n+1/2} = 1/2 sum_faces rho_f |v^{n+1/2}|^2
 *                           + 1/2 sum_cells p^{n+1} p^n / K,
 *   the staggered-time discrete energy, conserved exactly by the lossless
 *   scheme because the divergence is minus the transposed gradient
 *   (rho_f = mean density of the two cells of a face, K with the speed
 *   perturbation, beta not included);
 * out[3 d + 1] = max |p^{n+1}|;  out[3 d + 2] = number of non-finite p^{n+1}.
 * FP64 sums in a fixed order.  out is host double [n_domains][3].
 * Synchronises the stream.  Returns FW_ENONFINITE (out still filled) if any
 * pressure is NaN or infinite.  On first use the library allocates one
 * pressure-sized device buffer and one partial-sum buffer.
 */
int fw_energy_step(fw_sim *sim, double *out, void *hip_stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * step and diagnostics as fw_energy_step, with p^n and the partial sums kept
 * in a fixed scratch array inside the library (one per GPU, held until the
 * process ends) instead of buffers allocated on first use.  Calls no
 * allocating routine.  Limits: at most 8 Mi cells in all domains together
 * (domains padded to 64 cells) and 65536 marching tiles, else FW_EINVAL.
 * The tile lists must already exist (building them allocates): take one
 * fw_step or fw_energy_step first, else FW_ESTATE.  Every call on one GPU
 * uses that GPU's single scratch array, so calls that overlap on one GPU
 * (other host threads, other streams) race.  Synchronises the stream.
 */
int fw_energy_step_noalloc(fw_sim *sim, double *out, void *hip_stream);

/*
 * Copy one field of one domain (cells in the domain's linear order) to dst
 * (device memory if dst_is_device, else host): FW_FIELD_P the pressure,
 * FW_FIELD_VX/VY/VZ the velocity at faces i+1/2 (stored at cell i).
 * Synchronises the stream.
 */
enum { FW_FIELD_P = 0, FW_FIELD_VX = 1, FW_FIELD_VY = 2, FW_FIELD_VZ = 3 };
int fw_read_field(fw_sim *sim, int field, int domain, float *dst, int dst_is_device, void *hip_stream);

/*
 * Memory-traffic probe (measurement only; Sec. 3.3's step is bound by memory
 * bandwidth, and this measures what a schedule of it can reach): moves the
 * per-cell state streams of one 3D domain with none of the method's
 * arithmetic, writing every value back unchanged, reps times, and returns the
 * average milliseconds per pass in *avg_ms.
 *   mode 0: the velocity update's streams (p, class map, v and the 3N face
 *           memory variables read; v and the memory variables written);
 *   mode 1: the pressure update's (v, p, class map, N cell memory variables
 *           read; p and the memory variables written);
 *   mode 2: the whole state read and written once (a fused update's pass);
 *   mode 3: mode 0 with the three per-axis face memory-variable groups of a
 *           cell read and written as one [cell][axis][N] stream over the
 *           memory of the three arrays (a layout the step does not use;
 *           every address still gets back the value read from it);
 *   mode 4: mode 3 with v read and written as one [cell][axis] stream too;
 *   mode 5: mode 0 with the face memory variables blocked by 64 cells,
 *           [cell / 64][axis][cell % 64][N] (needs a multiple of 64 stored
 *           cells, FW_EUNSUPPORTED otherwise);
 *   mode 6: mode 5 with v blocked the same way, [cell / 64][axis][cell % 64].
 *   order 0: one flat sweep (neighbouring cells in concurrent workgroups);
 *   order 1: 64 x 4 tiles each marching 48 planes along z.
 * CPML variables are not moved.  Requires one 3D domain (FW_EUNSUPPORTED
 * otherwise) and fw_set_media.  Synchronises the stream.
 */
int fw_stream_probe(fw_sim *sim, int mode, int order, int reps, void *hip_stream, double *avg_ms);

/*
 * Infrastructure (no operation of the method).
 * Streaming device-to-device copy of bytes bytes on hip_stream (used for
 * state snapshots and checkpoints).  16-byte aligned pointers and sizes use a
 * kernel with one float4 per lane, launched in pieces of at most 16 GiB;
 * anything else hipMemcpyAsync.  Asynchronous.
 */
int fw_device_copy(void *d_dst, const void *d_src, int64_t bytes, void *hip_stream);

/*
 * Tuning and behaviour options (host only):
 *   FW_OPT_GRAPH_STEPS   steps per captured HIP graph (0 = eager only); default 16.
 *   FW_OPT_MARCH_CHUNK   cells of the marching axis per tile (>= 1); default auto
 *                        (3D: about 48 planes; 2D: 8 rows).
 *   FW_OPT_TILE_ROWS     3D tile rows along y per block: 4, 8 or 16; default 4.
 *   FW_OPT_ROWS_PER_THREAD  3D rows each thread owns: 1 or 2 (not with 4-row
 *                        tiles); default 1.
 *   FW_OPT_PERSISTENT    0: one workgroup per tile (default); k > 0: a
 *                        persistent grid of 32 k workgroups per XCD
 *                        (k per CU) that walk the tile list.
 *   FW_OPT_TILE_ORDER    order of the marching tiles: 0 = x fastest within a
 *                        chunk (default), 1 = y fastest, 2 = plane-major with
 *                        XCD k owning y-band k of every chunk (3D).
 *   FW_OPT_PLANE_KERNELS 3D: 1 or -1 (default) = both updates run on 64 x R
 *                        tiles of a few planes (FW_OPT_VEL_PLANES,
 *                        FW_OPT_PRS_PLANES), plane-major with XCD k owning
 *                        y-band k of every plane (the z stencil reads its
 *                        eight-plane window from memory: it stays in the
 *                        last-level cache); 0 = both march the tiles set by the
 *                        options above.
 *                        2D: 1 or -1 (default) = both updates run on 64 x R
 *                        tiles, one per block, with both stencils read from
 *                        LDS; 0 = both march along y.  Not used with a
 *                        persistent grid.
 *   FW_OPT_PLANE_ROWS    rows R of those tiles along y: 4 (3D default) or 8
 *                        (2D default); 16 in 2D.  More rows mean fewer y-halo
 *                        reads per cell; which is faster depends on the grid
 *                        (the autotuner times them).
 *   FW_OPT_STEP_CHUNK    3D with both plane kernels: C >= 4 = the step runs
 *                        the velocity update over planes [cC, (c+1)C) then the
 *                        pressure update over [cC-3, (c+1)C-3), chunk after
 *                        chunk (same results); 0 = each update runs once over
 *                        the whole grid; -1 (default) = 120-plane chunks on
 *                        grids of at least 320 planes of 100 k cells, whole-
 *                        grid launches otherwise.  fw_time_kernels follows
 *                        the same schedule; the energy step and the adjoint
 *                        run whole-grid launches.
 *   FW_OPT_VEL_PLANES    planes per tile of the velocity plane kernel: 1, 2
 *                        or 4 (more loads in flight per thread, more
 *                        registers); default 1 with N >= 3 mechanisms, 2 with
 *                        N <= 2.
 *   FW_OPT_PRS_PLANES    planes per tile of the pressure plane kernel: 2, 4
 *                        or 8 (a longer tile re-reads the v_z window less
 *                        often, a shorter one needs fewer registers); default
 *                        2 with N >= 3 mechanisms, 8 with N <= 2.
 *   FW_OPT_RESIDENT_1D   1D grids: -1 (default) or 1 = fw_step runs one
 *                        workgroup per domain that keeps the domain's state
 *                        on chip (p and v in LDS, memory variables in
 *                        registers) for up to 4096 steps per launch, when
 *                        every domain has at most 8192 cells, the two CPML
 *                        slabs at most 1024 cells together and no strength
 *                        map is set (otherwise, and with 0, the per-step
 *                        kernels).  fw_time_kernels, the energy step and the
 *                        adjoint's reverse sweep use the per-step kernels.
 * Options change the work decomposition only, never the results.
 */
enum { FW_OPT_GRAPH_STEPS = 1, FW_OPT_MARCH_CHUNK = 2, FW_OPT_TILE_ROWS = 3, FW_OPT_ROWS_PER_THREAD = 4,
       FW_OPT_PERSISTENT = 5, FW_OPT_TILE_ORDER = 6, FW_OPT_PLANE_KERNELS = 7, FW_OPT_PLANE_ROWS = 8,
       FW_OPT_VEL_PLANES = 9, FW_OPT_PRS_PLANES = 10, FW_OPT_STEP_CHUNK = 11, FW_OPT_RESIDENT_1D = 12 };
int fw_set_option(fw_sim *sim, int key, int64_t value);

#ifdef __cplusplus
}
#endif
#endif /* FW25_H */
