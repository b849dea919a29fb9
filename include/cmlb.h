/*
 * cmlb.h -- C-ABI of the MI355X (gfx950) library that advances the coupled pair
 * of D2Q9 cascaded central-moment lattice Boltzmann schemes of Hajabdollahi,
 * Premnath & Welch (arXiv:1909.04166):
 *
 *   - the pressure-based hydrodynamic scheme for gbar (Sec. 4) with the
 *     net-gradient pressure force F_p, the surface-tension force F_s (capillary and
 *     Marangoni terms, Eqs. surfacetensiongeometricsurfactantsxcomp/ycomp, or the
 *     chemical-potential form of Eq. surfacetensionthermodynamic) and a body force;
 *   - the conservative Allen-Cahn (phase-field) scheme for f (Sec. 5);
 *   - options used by the paper's test problems: the single-relaxation-time (SRT)
 *     pair of the stability comparison (Sec. 7), free-slip walls (Secs. 6.4, 6.5),
 *     the Langmuir surface-tension law of an imposed surfactant concentration
 *     (Eq. Langmuirisotherm, Sec. 6.7) and the phase field alone under an imposed
 *     velocity (Sec. 6.1);
 *   - the isotropic finite-difference fields that couple them (grad phi, n,
 *     div n, lap phi, chemical potential, grad rho, grad p; text after
 *     Eq. fluidviscosity).
 *
 * Conventions
 *   - Every function returns an lb_status: 0 on success, a negative code on error.
 *   - The library never allocates device memory.  The caller passes one device
 *     workspace (size from lb_workspace_bytes) and keeps it alive until
 *     lb_destroy / lb_batch_destroy.  The library allocates small host-side state
 *     (the handle, pinned host words for diagnostics).
 *   - All device work is ordered on the caller's HIP stream, passed as void*
 *     (a hipStream_t; NULL means the default stream).  Functions that return host
 *     data synchronize that stream; lb_step and lb_batch_step do not.
 *   - Host arrays of fields are FP64, row-major with index y*nx + x, whatever the
 *     storage precision.  Distribution arrays are FP64 [9][ny][nx] in the
 *     velocity order 0 rest, 1 +x, 2 +y, 3 -x, 4 -y, 5 (+,+), 6 (-,+), 7 (-,-),
 *     8 (+,-) (Eq. particlevelocities).
 *   - Node (x, y) = (i, j).  Each direction is periodic or bounded by walls at
 *     -1/2 and n - 1/2: halfway bounce-back (no slip) or halfway specular
 *     reflection (free slip).  A population whose source lies beyond an x and a
 *     y wall at once is bounced back.
 *   - A handle is not thread-safe; distinct handles are independent.
 */
#ifndef CMLB_H
#define CMLB_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t lb_status;
enum {
    LB_OK = 0,
    LB_E_INVALID_ARG = -1, /* a parameter is out of range, a pointer is NULL */
    LB_E_WORKSPACE = -2,   /* workspace too small or misaligned (256 B) */
    LB_E_HIP = -3,         /* a HIP runtime call failed */
    LB_E_UNSTABLE = -4,    /* a diagnostic found NaN/Inf or max|u| above the limit */
    LB_E_UNSUPPORTED = -5, /* a valid but unimplemented option */
    LB_E_STATE = -6,       /* buffer of the wrong size for save/load */
    LB_E_TOO_LARGE = -7    /* lattice beyond the static scratch of lb_step_noalloc */
};

enum { LB_PERIODIC = 0, LB_HALFWAY_BB = 1, LB_FREE_SLIP = 2 };
/* collision model of both schemes:
 *   LB_CASCADED          cascaded central moments (Secs. 4, 5); the hydrodynamic
 *                        moment changes h_3..h_8 solve the relaxation conditions
 *                        of Sec. 4 as stated (the incoming gbar's own central
 *                        moments, h_0..h_2 carried into the higher moments);
 *   LB_SRT               the single-relaxation-time comparison pair (Sec. 7; BGK
 *                        toward second-order Hermite equilibria and sources with
 *                        the same zeroth to second moments, one rate:
 *                        omega(nu(phi)) for gbar, omega^phi for f);
 *   LB_CASCADED_PRINTED  as LB_CASCADED with the printed closed forms of h_3..h_8
 *                        (Eq. cascadedcollisionoperator), which leave out both
 *                        effects above and differ by O(F) in h_6, h_7.
 * The phase-field cascade is the same in LB_CASCADED and LB_CASCADED_PRINTED. */
enum { LB_CASCADED = 0, LB_SRT = 1, LB_CASCADED_PRINTED = 2 };
/* LB_FLOW_IMPOSED: only the phase field f is advanced, under the velocity set by
 * lb_set_velocity (Sec. 6.1); gbar, the pressure and all forces are absent. */
enum { LB_FLOW_COUPLED = 0, LB_FLOW_IMPOSED = 1 };
/* surface-tension law: linear sigma(T(y)), or Langmuir
 * sigma = sigma0 (1 + beta ln(1 - psi)) of psi(y) = psi_a + psi_G y (geometric form only) */
enum { LB_SIGMA_LINEAR = 0, LB_SIGMA_LANGMUIR = 1 };
/* reference density of the body force F_ext = (rho - rho_ref) g */
enum { LB_FREF_MEAN = 0, LB_FREF_LIGHT = 1, LB_FREF_HEAVY = 2, LB_FREF_NONE = 3 };
/* surface-tension form: geometric with Marangoni term (default), or chemical potential */
enum { LB_ST_GEOMETRIC = 0, LB_ST_CHEMPOT = 1 };
/* storage precision of the 18 distribution planes; compute is FP64 for LB_FP64 and FP32 otherwise */
enum { LB_FP64 = 0, LB_FP32 = 1, LB_FP32_F16 = 2, LB_FP32_BF16 = 3 };
/* built-in initial phase field (lb_init_fields / lb_batch_add with phi0 = NULL): the
 * equilibrium profile phi0 = 1/2 + 1/2 tanh(2 d / W) of the conservative Allen-Cahn
 * equation (Sec. 2) of a signed distance d, positive in phase A:
 *   LB_INIT_DROPLET   init_par = {xc, yc, R, s, px, py}: d = s (R - r), r the distance
 *                     to (xc, yc); s = +1 a drop of phase A (Sec. 6.2), -1 a bubble of
 *                     phase B (Sec. 6.5); px, py > 0 repeat it with that period
 *                     (x and y taken modulo px, py first; 0: no repetition);
 *   LB_INIT_ELLIPSE   init_par = {xc, yc, a, b, px, py}: semi-axes a (x), b (y) of phase
 *                     A (Sec. 7); d = r (1/q - 1) with q = sqrt((X/a)^2 + (Y/b)^2), the
 *                     radial scaling of the ellipse (d = max(a, b) at the centre);
 *   LB_INIT_INTERFACE init_par = {y0, A, k}: phase A above y0 + A cos(2 pi k x / nx)
 *                     (Sec. 6.3 with k = 1; a flat interface with A = 0):
 *                     d = y - y0 - A cos(2 pi k x / nx).
 * Node (i, j) sits at (x, y) = (i, j). */
enum { LB_INIT_NONE = 0, LB_INIT_DROPLET = 1, LB_INIT_ELLIPSE = 2, LB_INIT_INTERFACE = 3 };
/* rounding of the values a step stores in 16-bit storage (LB_FP32_F16, LB_FP32_BF16;
 * ignored otherwise).  LB_ROUND_STOCHASTIC: each value is rounded up or down at
 * random with the probabilities that make it unbiased (the gfx950 conversions with
 * stochastic rounding), the random bits a hash of the step count, the node and the
 * direction, so that results do not depend on the schedule and repeat bit for bit.
 * With round to nearest, a change of a stored value below half its unit in the
 * last place is lost every step: a slowly moving interface (the thermocapillary
 * drop of Sec. 6.6 at about 3e-4 nodes per step) stays where it is.
 * Initial states, lb_set_dist and lb_load_state round to nearest. */
enum { LB_ROUND_STOCHASTIC = 0, LB_ROUND_NEAREST = 1 };

/*
 * Problem description (Secs. 2, 4, 5).  Phase A is phi = 1, phase B is phi = 0.
 *   rho(phi) = rho_B + phi (rho_A - rho_B), mu(phi) = mu_B + phi (mu_A - mu_B),
 *   mu_X = rho_X nu_X; omega_4 = omega_5 = 1 / (1/2 + 3 nu(phi)); other hydro rates 1.
 *   M = (1/omega^phi - 1/2) / 3 for the first-order ACE moments; other ACE rates 1.
 *   sigma(y) = sigma0 + sigma_T * (T0 + dTdy * (y - y_ref)), or the Langmuir law;
 *   kappa~ = 1.5 W sigma(y), its y derivative analytic.
 * Derived rates must lie in (0, 2); under the Langmuir law 1 - psi(y) > 0 on every row.
 */
typedef struct lb_config {
    int32_t nx, ny;          /* lattice size, each >= 8 */
    int32_t bc_x, bc_y;      /* LB_PERIODIC, LB_HALFWAY_BB or LB_FREE_SLIP in x and in y */
    int32_t force_ref;       /* LB_FREF_* */
    int32_t st_form;         /* LB_ST_* */
    int32_t precision;       /* LB_FP64, LB_FP32, LB_FP32_F16, LB_FP32_BF16 */
    int32_t diag_every;      /* >0: lb_step checks stability every diag_every steps */
    double rho_A, rho_B;     /* densities, > 0 */
    double nu_A, nu_B;       /* kinematic viscosities, > 0 */
    double sigma0, sigma_T;  /* surface tension law */
    double T0, dTdy, y_ref;  /* imposed linear temperature T(y) */
    double W, M;             /* interface width (> 0) and mobility (> 0) */
    double gx, gy;           /* body-force acceleration */
    double shift_f, shift_g; /* 16-bit storage stores f_a - w_a shift_f and g_a - w_a shift_g.
                                Recommended: shift_f the light phase's phi (0 when rho_A >=
                                rho_B, else 1), whose values are then stored near zero where
                                rho(phi) is most sensitive to phi, and shift_g 0 */
    double u_max;            /* stability limit for diagnostics (0: 0.3) */
    int32_t tile_x;          /* workgroup width in lanes: 64, 128, 132, 256, 260, 452, 512,
                                516, or 1024 (FP32-compute
                                precisions without prefetching); strips of tile_x - 4
                                columns; 0: autotuned */
    int32_t tile_h;          /* rows per work item (>= 1); 0: autotuned (lattices under
                                65536 nodes: one item per workgroup, rows halved until
                                there are two items per CU, prefetching) */
    int32_t collision;       /* LB_CASCADED or LB_SRT */
    int32_t flow;            /* LB_FLOW_COUPLED or LB_FLOW_IMPOSED */
    int32_t surf;            /* LB_SIGMA_LINEAR or LB_SIGMA_LANGMUIR */
    int32_t tile_pf;         /* with tile_x and tile_h both set: 1 selects the kernel
                                variant that prefetches the next rows during the
                                collision (LB_CASCADED with LB_FLOW_COUPLED only);
                                must be 0 otherwise */
    double beta, psi_a, psi_G; /* Langmuir law parameters */
    int32_t init_kind;       /* LB_INIT_*: the built-in initial phase field */
    int32_t rounding;        /* LB_ROUND_*: rounding of 16-bit stores (0: stochastic) */
    double init_par[8];      /* its parameters (see LB_INIT_*) */
} lb_config;

typedef struct lb_diag {
    double step;       /* time step of the state */
    double sum_phi;    /* sum over nodes of phi */
    double sum_rho;    /* sum over nodes of rho(phi) */
    double max_u;      /* max |u| (NaN if any |u| is NaN) */
    double dp_laplace; /* p(nx/2, ny/2) - p(0, 0) (Laplace-Young probe, Sec. 6.2) */
    double r_eff;      /* sqrt(sum phi / pi) */
    double spike_y;    /* lowest phi = 1/2 crossing on column nx/2 (NaN if none) */
    double bubble_y;   /* highest phi = 1/2 crossing on column 0 (NaN if none) */
    double centroid_y; /* sum y phi / sum phi */
    double nan_flag;   /* 1 if any phi, p or u is NaN/Inf */
} lb_diag;

typedef struct lb_handle lb_handle;
typedef struct lb_batch lb_batch;

/* Static string for a status code. */
const char* lb_status_string(lb_status s);

/* Device workspace bytes for one lattice (two copies of the 18 planes in the
 * storage precision, four FP64 field planes, diagnostics and the work list; with
 * LB_FLOW_IMPOSED also two velocity planes in the compute type).
 * Errors: LB_E_INVALID_ARG. */
lb_status lb_workspace_bytes(const lb_config* cfg, uint64_t* bytes);

/* Validates cfg, lays the lattice out in dev_ws (device memory, 256-byte aligned,
 * at least lb_workspace_bytes), picks the tile shape and returns a handle.  The
 * parameters are the paper's problem statement: the two phases' densities and
 * viscosities with rho(phi), mu(phi) and omega(nu) of Eqs.
 * sfluidpropertiesinterpolation and fluidviscosity (Secs. 2, 4), the surface
 * tension kappa~ = 1.5 W sigma of the geometric form (Eq. surfacetensiongeometric
 * and its surfactant extension, Sec. 6.7), the interface width W and mobility M of
 * the conservative Allen-Cahn equation (Sec. 2; omega^phi of Sec. 5), a body force
 * (Secs. 6.3-6.5) and the boundary kinds.  The state is undefined until
 * lb_init_fields or lb_load_state / lb_set_dist.
 * Errors: LB_E_INVALID_ARG, LB_E_WORKSPACE, LB_E_HIP. */
lb_status lb_create(const lb_config* cfg, void* dev_ws, uint64_t ws_bytes, void* stream,
                    lb_handle** out);

/* Initial state at t = 0: f_a = w_a phi0, gbar_a = 0, i.e. p = 0 and u = 0 (the
 * paper states no initialization; this is the zero-velocity, zero-pressure
 * equilibrium of both schemes without the sharpening term, Secs. 4 and 5).
 * phi0: host, ny*nx FP64, caller-owned, read before return; or NULL for the
 * built-in field of cfg.init_kind, computed on the device (LB_E_INVALID_ARG if
 * init_kind is LB_INIT_NONE).  Synchronizes. */
lb_status lb_init_fields(lb_handle* h, const double* phi0);

/* Imposed velocity for LB_FLOW_IMPOSED (Sec. 6.1): host FP64 ux, uy of ny*nx each,
 * caller-owned, read before return; kept in the compute precision until replaced
 * (e.g. negated to reverse the flow).  Not part of a checkpoint.  Synchronizes.
 * Errors: LB_E_INVALID_ARG (NULL, or a coupled lattice). */
lb_status lb_set_velocity(lb_handle* h, const double* ux, const double* uy);

/* Advances n time steps.  One step (Secs. 4 and 5): the coupling fields at time t
 * (phi, pbar, grad phi, n, div n or the chemical potential, rho, F_s, F_t, u,
 * F_p, p; Eqs. netgradientpressureforce, hydrodynamicfields), the cascaded
 * collision of gbar with its sources (Eqs. cascadedcollisionoperator,
 * cumulativesourcetermcomponents, postcollisioncascadedLBscheme) and of f
 * (Sec. 5), then streaming with the boundary rules (Eq. ACEstreamingLB).
 * Enqueued asynchronously on the handle's stream.  With diag_every > 0, a
 * stability check runs every diag_every steps; LB_E_UNSTABLE is returned by the
 * first call after a check has found NaN/Inf or max|u| > u_max. */
lb_status lb_step(lb_handle* h, int64_t n);

/* phi (Sec. 5, zeroth moment of f), p and u (Eq. hydrodynamicfields) at the
 * current time.  Host buffers of ny*nx FP64; NULL skips a field.  Synchronizes. */
lb_status lb_get_fields(lb_handle* h, double* phi, double* p, double* ux, double* uy);

/* Writes the coupling fields at the current time into a caller-owned DEVICE
 * buffer of 9*ny*nx FP64: grad phi x, grad phi y, n_x, n_y, div n, F_t x, F_t y,
 * F_p x, F_p y.  For diagnosis of parity failures.  Synchronizes. */
lb_status lb_get_coupling(lb_handle* h, double* dev_out);

/* FP64 diagnostics at the current time (sums in a fixed order): total phase sum
 * phi (conserved by the Allen-Cahn scheme, Sec. 5), total mass, max |u|, the
 * Laplace probe p(centre) - p(corner) and R_eff = sqrt(sum phi / pi) (Sec. 6.2),
 * the spike and bubble tips (Sec. 6.3: phi = 1/2 crossings at the centre and edge
 * columns) and the centroid y (Secs. 6.4-6.7).  Synchronizes. */
lb_status lb_diagnostics(lb_handle* h, lb_diag* out);

/* Post-streaming distributions f, gbar at the current time (FP64 host arrays of
 * 9*ny*nx each; NULL skips one; gbar is all zero under LB_FLOW_IMPOSED).
 * Synchronizes. */
lb_status lb_get_dist(lb_handle* h, double* f, double* g);

/* Sets the state at time `step` from post-streaming FP64 distributions (host,
 * 9*ny*nx each), rounded to the storage precision.  g is ignored (and may be
 * NULL) under LB_FLOW_IMPOSED.  Synchronizes. */
lb_status lb_set_dist(lb_handle* h, const double* f, const double* g, int64_t step);

/* Bytes of a checkpoint: the 18 stored planes in the storage precision plus the
 * step counter.  save/load copy them to/from a caller-owned host buffer; a
 * resumed run is bit-identical.  Errors: LB_E_STATE on a size mismatch. */
lb_status lb_state_bytes(lb_handle* h, uint64_t* bytes);
lb_status lb_save_state(lb_handle* h, void* host, uint64_t bytes);
lb_status lb_load_state(lb_handle* h, const void* host, uint64_t bytes);

/* Current step counter. */
lb_status lb_get_step(lb_handle* h, int64_t* step);

/* Frees host-side state.  The workspace stays the caller's. */
void lb_destroy(lb_handle* h);

/* ------------------------------------------------------------------ batch ----
 * Many independent lattices of uneven sizes, each advanced by the step of
 * lb_step (Secs. 4, 5), by ONE persistent kernel launch per step over a shared
 * work list of (instance, strip, rows) items.  The paper runs one lattice at a
 * time; batching is this library's (the problem statement of each slot is an
 * lb_config, as for lb_create).
 * All instances share the storage precision, the collision model and one tile
 * shape; LB_FLOW_IMPOSED lattices are not batched.  A slot holds one lattice; slots can be filled and emptied between
 * steps (continuous batching).  Results of a slot do not depend on the other
 * slots (bit-identical to the same lattice alone). */

/* Workspace bytes for a batch with `slots` slots whose lattices are the
 * largest that fit in `node_capacity` nodes in total.
 * Errors: LB_E_INVALID_ARG. */
lb_status lb_batch_workspace_bytes(int32_t slots, int64_t node_capacity, int32_t precision,
                                   uint64_t* bytes);

/* Creates an empty batch over dev_ws.  tile_x / tile_h as in lb_config (0: defaults).
 * Unlike lb_create the batch is sized by slots and a node capacity, not by one
 * lattice: lattices are added and removed later (continuous batching), so the
 * workspace holds a pool from which each slot takes its two buffers. */
lb_status lb_batch_create(int32_t slots, int64_t node_capacity, int32_t precision,
                          int32_t tile_x, int32_t tile_h, void* dev_ws, uint64_t ws_bytes,
                          void* stream, lb_batch** out);

/* Places a lattice in a free slot and initializes it like lb_init_fields (phi0 NULL:
 * the built-in field of cfg->init_kind).
 * Returns the slot index in *slot.  A slot holds at most min(node_capacity,
 * 2^24) nodes.  Errors: LB_E_INVALID_ARG (bad config, or a precision or collision
 * model other than the batch's), LB_E_UNSUPPORTED (LB_FLOW_IMPOSED),
 * LB_E_WORKSPACE (no free slot, not enough free nodes, or lattice too large).
 * Synchronizes. */
lb_status lb_batch_add(lb_batch* b, const lb_config* cfg, const double* phi0, int32_t* slot);

/* Frees a slot (its storage is reused by later adds). */
lb_status lb_batch_remove(lb_batch* b, int32_t slot);

/* Advances every occupied slot by n steps: n launches of the persistent
 * kernel.  With use_graph != 0, once the batch's lattices have not changed
 * (add / remove) for 128 steps, whole runs of 32 steps are replayed from
 * captured HIP graphs; the steps of a call up to that point, and the remainder
 * below 32, are launched one by one.  Asynchronous. */
lb_status lb_batch_step(lb_batch* b, int64_t n, int32_t use_graph);

/* Pins the batch's schedule as lb_set_schedule does for one lattice (mode 2 over
 * lattices of different heights is cut as mode 1); the autotuner no longer runs.
 * Synchronizes the stream and drops captured graphs.  Errors: LB_E_INVALID_ARG
 * (an invalid value or a cut that does not fit the work-list capacity; the
 * previous schedule then stays). */
lb_status lb_batch_set_schedule(lb_batch* b, int32_t tile_x, int32_t mode, int32_t param, int32_t prefetch);

/* Steps the batch has replayed from captured graphs and launched one by one
 * since it was created. */
lb_status lb_batch_launch_counts(lb_batch* b, int64_t* graph_steps, int64_t* eager_steps);

/* Fields / diagnostics / step of one slot, as for a single lattice. Synchronize. */
lb_status lb_batch_get_fields(lb_batch* b, int32_t slot, double* phi, double* p, double* ux,
                              double* uy);
lb_status lb_batch_diagnostics(lb_batch* b, int32_t slot, lb_diag* out);
lb_status lb_batch_get_step(lb_batch* b, int32_t slot, int64_t* step);

/* Number of occupied slots and nodes in use. */
lb_status lb_batch_usage(lb_batch* b, int32_t* used_slots, int64_t* used_nodes);

void lb_batch_destroy(lb_batch* b);

/* ------------------------------------------------------------- measurement ---
 * Average duration in milliseconds of the fused step kernel over the last
 * lb_step / lb_batch_step call that enabled timing (HIP events on the handle's
 * stream around the kernel launches).  timing_enable(1) before the step call,
 * read after synchronizing. */
lb_status lb_timing_enable(lb_handle* h, int32_t on);
lb_status lb_timing_read(lb_handle* h, double* ms_per_step, int64_t* steps);
lb_status lb_batch_timing_enable(lb_batch* b, int32_t on);
lb_status lb_batch_timing_read(lb_batch* b, double* ms_per_step, int64_t* steps);

/* Pins the handle's schedule; later steps skip the autotuner.  tile_x as in
 * lb_config; mode 0: work items of `param` rows (>= 1), one per workgroup;
 * mode 1: persistent grid of param (1..4) x resident workgroups per CU x CUs,
 * each workgroup one balanced run of the concatenated strip rows; mode 2: as 1,
 * the grid cut down to strips x bands (bands a multiple of 8) so that every
 * strip is cut at the same rows and the same rows of neighbouring strips run on
 * one XCD.  prefetch as lb_config.tile_pf.  The step results do not depend on the
 * schedule (bit for bit).  Synchronizes the handle's stream (the work list is
 * uploaded from the host) and drops captured step graphs.  Returns
 * LB_E_INVALID_ARG for an invalid value or a cut that does not apply to the
 * lattice (too few rows for the bands); the previous schedule then stays. */
lb_status lb_set_schedule(lb_handle* h, int32_t tile_x, int32_t mode, int32_t param, int32_t prefetch);
/* Schedule chosen for the handle (after autotuning when tile_x/tile_h were 0):
 * workgroup width tile_x (lanes; the strip is tile_x - 4 columns), rows per work
 * item (or per persistent segment), the persistent grid size (0 when every work
 * item gets its own workgroup) and whether the kernel variant that prefetches
 * the next rows during the collision is used (1) or not (0). */
lb_status lb_get_schedule(lb_handle* h, int32_t* tile_x, int32_t* rows, int32_t* grid,
                          int32_t* prefetch);
/* The same for a batch: the schedule of its persistent step (rows is the segment
 * length; 0 until the batch has stepped with at least one occupied slot). */
lb_status lb_batch_get_schedule(lb_batch* b, int32_t* tile_x, int32_t* rows, int32_t* grid,
                                int32_t* prefetch);

/* ------------------------------------------------------- no allocation ----
 * For callers that cannot allocate memory: code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc.  Advances one lattice by n
 * steps (the same step as lb_step) without a handle or a workspace and without
 * allocating anything, host or device.
 *
 *   cfg            as for lb_create; LB_FLOW_COUPLED only and diag_every = 0
 *                  (LB_E_UNSUPPORTED otherwise).  tile_x / tile_h / tile_pf are
 *                  honoured; 0 takes a fixed default schedule (no autotuning).
 *   state0, state1 caller-owned DEVICE buffers, 256-byte aligned, state_bytes each
 *                  (at least the checkpoint size of lb_state_bytes minus its 16-byte
 *                  header): the 18 stored planes in the storage precision, in the
 *                  layout lb_save_state writes after that header.  The current
 *                  state is read from state0; after the call it is in state0 if n
 *                  is even and in state1 if n is odd.
 *   step           step count of the state in state0 (as lb_get_step reports it for
 *                  a handle); it seeds the stochastic rounding of 16-bit storage, so
 *                  the same step count gives the same bits as lb_step.
 *   stream         HIP stream (void*); every launch is enqueued there and the
 *                  call returns without synchronizing.  It makes no copy, memset or
 *                  synchronization, so it can be captured into a HIP graph once a
 *                  first call on the device has looked up the scratch address.
 *
 * The descriptor, step counter, work list and per-row table live in a static 1 MiB device
 * array that each GPU holds until the process ends; it must hold the work list
 * (16 bytes per (strip, row block)) and, under the Langmuir law, 16 ny bytes:
 * larger lattices (or tiles that cut them finer) return LB_E_TOO_LARGE before any
 * device work.  Calls on one GPU share that array: calls that overlap on one
 * device (other streams or threads) race and must be serialized by the caller.
 * Errors: LB_E_INVALID_ARG, LB_E_UNSUPPORTED, LB_E_WORKSPACE (buffers too small
 * or misaligned), LB_E_TOO_LARGE, LB_E_HIP. */
lb_status lb_step_noalloc(const lb_config* cfg, void* state0, void* state1, uint64_t state_bytes,
                          int64_t step, int64_t n, void* stream);

/* sizeof(lb_config) and sizeof(lb_diag) as compiled, for binding checks. */
lb_status lb_struct_sizes(uint64_t* config_bytes, uint64_t* diag_bytes);

/* Device-to-device copy kernel over n bytes (attainable-bandwidth reference for
 * the roofline).  Enqueued on `stream`; src/dst are device pointers, 16-byte aligned. */
lb_status lb_copy_kernel(void* dst, const void* src, uint64_t n, void* stream);

/* Streams bounding the attainable HBM bandwidth, n bytes (>= 16 MiB, a multiple
 * of 16), device pointers 16-byte aligned, enqueued on `stream`:
 *   0 the copy of lb_copy_kernel (4 x 16 B per lane in flight);
 *   1 copy, persistent grid (16 workgroups per CU), 8 x 16 B per lane in flight;
 *   2 as 1 with nontemporal loads and stores;  3 as 1 with 4 in flight and
 *     nontemporal stores;  4 copy, one contiguous chunk per workgroup;
 *   5 read only: reads src, writes one 16-byte word per lane of the grid to dst
 *     (16 MiB);  6 write only: fills dst;
 *   7 the step kernel's memory pattern in 16-bit storage without its arithmetic:
 *     whole rows of 18 planes of 8064 two-byte values (the first
 *     floor(n / 290304) rows), 18 strips of 448 columns x 28 row segments, each
 *     lane loading its 18 values of a row and storing them, one column per lane
 *     with 2-byte accesses;  8 as 7 with two columns per lane and 4-byte accesses.
 * Errors: LB_E_INVALID_ARG. */
lb_status lb_bandwidth_probe(void* dst, const void* src, uint64_t n, int32_t variant, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* CMLB_H */
