/*
 * lbm_ms.h - C ABI of the MI355X (gfx950) library for the advection-diffusion lattice Boltzmann
 * model coupled to the Maxwell-Stefan equations (Huang, Bao, Jiang, Zhang, arXiv 1809.01600).
 *
 * The problem is the paper's anode of Section 4.1: a porous voxel domain, x = diffusion direction,
 * a Dirichlet (channel-side) inlet at x = 0, a reactive-flux outlet at the anode/electrolyte
 * interface x = nx - 1, periodic in y and z.  Species 1 (H2) and 2 (H2O) carry populations; the
 * inert species 3 (Ar) is the balance X_3 = 1 - X_1 - X_2 (the (n-1)-dimensional closure of
 * Section 3.2).  One step is, per fluid node: pull-stream of the post-collision populations with
 * half-way bounce-back on solid links (Section 3.3), the inlet and outlet rules, the moments, the
 * gradients (Eq. 35 / Eq. 37 / central differences), the Maxwell-Stefan flux solve (Eq. 31-34,
 * Gamma = I), the effective diffusivity (Eq. 24 with signed flux norms), the relaxation time
 * (Eq. 25) and the BGK collision toward w_a X (Eq. 28-29).
 *
 * Conventions
 *  - Every function returns an lbm_ms_status (0 = OK, < 0 = error) unless stated otherwise; no
 *    C++ exception crosses the ABI.  After an error, lbm_ms_last_error() describes it.
 *  - Device memory: the caller allocates one device buffer of lbm_ms_workspace_bytes() bytes and
 *    owns it; the handle never frees it.  The handle owns only host metadata and a small pinned
 *    host staging buffer.
 *  - Ordering: every call is ordered on params.stream (a hipStream_t, NULL = legacy default
 *    stream).  Calls that return host values synchronize that stream; lbm_ms_step does not.
 *  - Threading: a handle is used from one host thread at a time.
 *  - Units: SI at the ABI (T in K, p in Pa, D in m^2/s, dx in m, current density in A/m^2).
 *  - Arrays: node index n = (z * ny + y) * nx + x (x fastest).  Field arrays are [3][N] float64
 *    (species-major), population arrays [2][Q][N] float64.
 */
#ifndef LBM_MS_H
#define LBM_MS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_ms_s* lbm_ms_t;

typedef enum {
    LBM_MS_OK = 0,
    LBM_MS_E_ARG = -1,          /* invalid argument (sizes, compositions, null pointers) */
    LBM_MS_E_STATE = -2,        /* call out of order (e.g. step before set_geometry/init) */
    LBM_MS_E_GEOM = -3,         /* no fluid path links the inlet column to the outlet column */
    LBM_MS_E_HIP = -4,          /* HIP runtime error (message in lbm_ms_last_error) */
    LBM_MS_E_DIVERGED = -5,     /* non-finite mole fraction found by a residual check */
    LBM_MS_E_NOT_CONVERGED = -6,/* max_steps reached before the residual fell below tol */
    LBM_MS_E_NEG_FRACTION = -7, /* a mole fraction below -1e-12 (limiting current exceeded) */
    LBM_MS_E_NOMEM = -8,        /* workspace too small, or host allocation failed */
    LBM_MS_E_TAU_CLAMP = -9     /* a relaxation time hit tau_min / tau_max since the last check */
} lbm_ms_status;

/* velocity sets, all with c_s^2 = 1/3 (Sec. 3.1): D2Q9; D3Q19; D2Q5 (rest 1/3, axis links 1/6);
 * D3Q7 (rest 0, axis links 1/6) */
enum { LBM_MS_D2Q9 = 0, LBM_MS_D3Q19 = 1, LBM_MS_D2Q5 = 2, LBM_MS_D3Q7 = 3 };

/* population storage (collision arithmetic is FP64 for LBM_MS_FP64, FP32 otherwise; the
 * Maxwell-Stefan solve, residual, mass balance and overpotential are FP64 in every mode) */
enum { LBM_MS_FP64 = 0, LBM_MS_FP32 = 1, LBM_MS_FP16 = 2, LBM_MS_BF16 = 3 };

/* 16-bit storage holds f - w_a c: c = inlet composition (GLOBAL) or the node's own mole
 * fraction, kept in an FP32 field (NODE) */
enum { LBM_MS_SHIFT_GLOBAL = 0, LBM_MS_SHIFT_NODE = 1 };

/* flux-norm ratio |N_j| / |N_i| in Eq. 24: from the local generalized-Fick fluxes (LOCAL_FLUX,
 * the paper's reading) or fixed at the stoichiometric ratio |nu_j| / |nu_i| (STOICH) */
enum { LBM_MS_LOCAL_FLUX = 0, LBM_MS_STOICH = 1 };

/* x = 0 face: Dirichlet anti-bounce-back (Eq. 36) or a bounce-back wall (closed box) */
enum { LBM_MS_INLET_DIRICHLET = 0, LBM_MS_INLET_WALL = 1 };

/* Collision: the paper's BGK (Eq. 28), or two relaxation times (TRT): the odd part of each link
 * pair relaxes with the Eq. 25 tau, which keeps setting the diffusivity, and the even part with
 * tau_even = 1/2 + Lambda / (tau - 1/2).  With Lambda fixed, steady states in resolved porous
 * media no longer depend on tau_ref (BGK's bounce-back walls move with tau). */
enum { LBM_MS_BGK = 0, LBM_MS_TRT = 1 };

typedef struct {
    int lattice;          /* LBM_MS_D2Q9, LBM_MS_D2Q5 (2D, nz = 1; also for batches), or
                             LBM_MS_D3Q19, LBM_MS_D3Q7 (3D) */
    int nx, ny, nz;       /* nodes; nz must be 1 for the 2D sets; nx >= 2 */
    double T;             /* K */
    double p;             /* Pa; C_t = p / (R T), R = 8.3145 */
    double D[9];          /* binary Maxwell-Stefan diffusivities D_ij [m^2/s], row-major 3x3,
                             symmetric, diagonal ignored */
    int nu[3];            /* stoichiometric coefficients (Eq. 39); need nu1 = -nu2 != 0, nu3 = 0,
                             or with advection nu1 != 0, nu2 != 0, nu3 = 0 and the 1D flux ratios
                             finite: -nu_s and -nu_s + nu1 + nu2 nonzero and of one sign, s = 1, 2 */
    int n_electrons;      /* electrons per reaction (Eq. 39, Eq. 43) */
    double dx;            /* lattice spacing [m] */
    double tau_ref;       /* dt = (tau_ref - 1/2) dx^2 / (3 max D_ij): the fastest binary pair
                             relaxes with tau_ref (c_s^2 = 1/3, Eq. 25) */
    int precision;        /* LBM_MS_FP64 / FP32 / FP16 / BF16 */
    int shift_mode;       /* LBM_MS_SHIFT_GLOBAL / NODE (16-bit storage only) */
    int ms_mode;          /* LBM_MS_LOCAL_FLUX / LBM_MS_STOICH */
    int inlet_mode;       /* LBM_MS_INLET_DIRICHLET / LBM_MS_INLET_WALL */
    double eps_flux;      /* regularizer of the flux-norm ratio, lattice units; < 0 selects
                             1e-2 * max|Q_s| + 1e-14 (set at lbm_ms_set_bc) */
    double tau_min;       /* relaxation-time clamp; 0 selects 0.5 + 1e-9 */
    double tau_max;       /* 0 selects 1e6 */
    int tile_y;           /* launch shape (0 = default); see lbm_ms_tile_options */
    int chunk_z;          /* 3D: planes per workgroup (0 = default).  2D: the row limit of packed
                             tiles (see lbm_ms_tile_options); 0 = default, which is 12 (packed)
                             when tile_y is 8 and fixed 64 x tile_y tiles otherwise */
    void* stream;         /* hipStream_t */
    int collision;        /* LBM_MS_BGK (0, the paper's) or LBM_MS_TRT */
    double trt_lambda;    /* TRT Lambda = (tau_even - 1/2)(tau - 1/2); <= 0 selects 1/4 */
    int advection;        /* 1: advective coupling (Sec. 3.1, Eq. 20-21 and 26) for reactions that
                             change the number of moles, nu1 + nu2 != 0: the species equilibrium
                             carries the molar-averaged velocity u_M = N_t / C_t of a second
                             lattice Boltzmann model (Stokes limit of an incompressible model with
                             the total concentration as density; no-slip on solid, inlet at the
                             channel's concentration, the electrode's total molar flux at each open
                             outlet node), the species see the mean u_M of the current and the
                             previous step, and Eq. 24 takes the diffusive fluxes J_s = N_s - X_s N_t
                             (Eq. 20) with J_j / J_i read as the projection of the vectors,
                             regularized toward the 1D steady ratio (-nu_j - X_j Nt) / (-nu_i - X_i
                             Nt), Nt = -(nu1 + nu2), which is also the STOICH variant.  Single
                             instances with FP64 or FP32 global storage, BGK, Dirichlet inlet, no
                             volumetric source and no checkpoints (E_ARG / E_STATE otherwise).
                             0: the equimolar method (Eq. 29), which needs nu1 = -nu2. */
    double tau_flow;      /* relaxation time of the velocity model (> 1/2; <= 0 selects 1) */
} lbm_ms_params;

typedef struct {
    double dt;            /* physical time step [s] */
    double Ct;            /* total molar concentration [mol/m^3] */
    double Dl[9];         /* lattice diffusivities D*_ij = D_ij dt / dx^2 */
    double Q[2];          /* lattice outflow per open outlet node per step, species 1 and 2 */
    double eps_flux;      /* regularizer in use */
    int64_t n_fluid;      /* fluid nodes after the connectivity clean-up */
    int64_t n_open_outlet;/* fluid nodes of the outlet column */
    int64_t steps;        /* steps taken since the last init */
    int q;                /* velocities of the lattice */
    int tile_x, tile_y, chunk_z; /* launch shape in use */
    size_t workspace_bytes;
    double S[2];          /* volumetric source per fluid node and step, species 1 and 2 ... */
    int64_t n_source;     /* ... on these fluid nodes ... */
    int source_x0;        /* ... of the columns x >= source_x0 (nx: no source) */
} lbm_ms_info;

/* Device bytes the caller must provide for these parameters (0 if the parameters are invalid). */
size_t lbm_ms_workspace_bytes(const lbm_ms_params* params);

/* Create a handle over caller-owned device memory d_workspace (at least
 * lbm_ms_workspace_bytes bytes, 256-byte aligned).  *out is NULL on error. */
int lbm_ms_create(const lbm_ms_params* params, void* d_workspace, size_t bytes, lbm_ms_t* out);

/* Solid mask on the host, nx*ny*nz bytes (1 = solid).  Fluid that no chain of lattice links
 * (periodic in y and z) connects to the inlet column becomes solid; E_GEOM when no fluid node of
 * the outlet column remains.  The fluid index map of the cleaned mask goes to the device.
 * In LBM_MS_INLET_WALL mode the mask is used as given.
 * Size limit: the kernels address each population buffer (2 species x Q links x P elements of
 * the storage type, P = fluid nodes rounded up to 64, plus 192) with 32-bit byte offsets, so
 * E_ARG when it would exceed 4 GiB: about 28.2 M fluid nodes for D3Q19 FP32, 14.1 M for FP64,
 * 56.5 M for 16-bit storage (D2Q9: 59.6 M, 29.8 M, 119 M; D3Q7: 76.7 M, 38.3 M, 153 M); with
 * the NODE shift also at most 268 M fluid nodes.  lbm_ms_workspace_bytes rejects boxes of more
 * than 2^30 voxels. */
int lbm_ms_set_geometry(lbm_ms_t h, const uint8_t* solid_host);

/* The same clean-up on the host only (no device, no handle): solid_out = cleaned mask,
 * *n_open = fluid nodes left in the outlet column (0: the outlet is unreachable). */
int lbm_ms_clean_geometry(int lattice, int nx, int ny, int nz, const uint8_t* solid_in,
                          uint8_t* solid_out, int64_t* n_open);

/* Cleaned mask (after set_geometry) copied to a host buffer of nx*ny*nz bytes. */
int lbm_ms_get_geometry(lbm_ms_t h, uint8_t* solid_host);

/* Boundary data: inlet mole fractions X_in[3] (>= 0, sum 1 within 1e-12) for the Dirichlet rule
 * (Eq. 36) and the current density j [A/m^2] (>= 0) of the electrode flux N_s = -nu_s j / (n F)
 * (Eq. 39).  Per open outlet node the lattice flux is Q_s = N_s dt / (C_t dx) * (ny nz / open
 * outlet nodes), so the outlet face carries the superficial current.  Call after set_geometry. */
int lbm_ms_set_bc(lbm_ms_t h, const double X_in[3], double j_A_per_m2);

/* Volumetric source (Eq. 27, F_a = w_a S_s): the reaction spread uniformly over the fluid nodes of
 * the columns x >= x_first, a functional layer next to the electrolyte, instead of (or besides)
 * the electrode flux at the outlet face.  The layer's total per step equals the electrode flux
 * of Eq. 39 at current density j [A/m^2] over the whole face, so per fluid node of the layer
 * S_s = -N_s dt n_face / (C_t dx n_layer) with N_s = -nu_s j / (n F): H2 is consumed, H2O made.
 * For reaction in the layer alone, give the outlet j = 0 in lbm_ms_set_bc (a closed face).
 * Set it before lbm_ms_init: the stored state is post-collision, so init places the first
 * collision's source on the layer, and the read-back of fields, outlet means and inventory
 * reports the mole fractions before each step's source, as the streamed state holds them.
 * x_first = nx removes the source; lbm_ms_set_geometry clears it.  E_ARG for x_first outside
 * [0, nx], j < 0, or a layer without fluid; E_STATE before lbm_ms_set_geometry.  Not for batch
 * members (their argument tables are set at lbm_ms_batch_create). */
int lbm_ms_set_source(lbm_ms_t h, int x_first, double j_A_per_m2);

/* Initial state f_a = w_a X0 (equilibrium).  X0 == NULL: uniform inlet composition.  Otherwise
 * X0 holds [3][N] float64 mole fractions (species 3 is ignored), in host memory
 * (x0_on_device = 0) or device memory (x0_on_device = 1).  Resets the step counter and the
 * residual snapshot. */
int lbm_ms_init(lbm_ms_t h, const double* X0, int x0_on_device);

/* The paper's initial field (Section 4.1): along x the flux equals the electrode flux and the
 * generalized Fick law (Eq. 31, Gamma = I) is integrated from the inlet composition; the 1D
 * profile is copied over y and z.  Uses the superficial flux (no open-area scaling). */
int lbm_ms_init_paper_profile(lbm_ms_t h);

/* The one-dimensional profile behind lbm_ms_init_paper_profile, prof[2][nx] (X_1, X_2 at the
 * node columns x = 0 .. nx - 1), copied to host memory.  Does not change the state. */
int lbm_ms_paper_profile(lbm_ms_t h, double* prof_host);

/* nsteps time steps, enqueued on the stream (asynchronous). */
int lbm_ms_step(lbm_ms_t h, int64_t nsteps);

/* nsteps steps bracketed by HIP events on the stream; *ms = elapsed milliseconds (synchronizes). */
int lbm_ms_time_steps(lbm_ms_t h, int64_t nsteps, double* ms);

/* Residual over the window since the previous snapshot (init or the last residual call):
 * r = ||X^t - X^{t-K}||_2 / (K ||X^t||_2) over fluid nodes and species 1, 2, K = steps since
 * the snapshot (FP64 accumulation).  Takes a new snapshot.  Returns E_DIVERGED for non-finite
 * values, E_NEG_FRACTION for X < -1e-12, E_TAU_CLAMP if a relaxation time was clamped. */
int lbm_ms_residual(lbm_ms_t h, double* residual);

/* Step until the residual, checked every check_every steps, is below tol, or max_steps steps
 * were taken (E_NOT_CONVERGED).  Error codes as lbm_ms_residual. */
int lbm_ms_converge(lbm_ms_t h, double tol, int64_t max_steps, int check_every,
                    int64_t* steps_taken, double* residual);

/* Mean mole fractions over the open outlet-column nodes (X_out[3], FP64). */
int lbm_ms_outlet_mean(lbm_ms_t h, double X_out[3]);

/* Concentration overpotential (Eq. 43): eta = (R T / n F) ln(X1_in X2_out / (X1_out X2_in)),
 * X_out = outlet_mean, in volts. */
int lbm_ms_overpotential(lbm_ms_t h, double* eta_volts);

/* Mole-fraction field of the current state.  X: [3][N] float64 in host memory (on_device = 0)
 * or device memory (on_device = 1); solid nodes read 0. */
int lbm_ms_get_fields(lbm_ms_t h, double* X, int on_device);

/* Advective coupling only: the molar-averaged velocity u_M that the species see (the mean of the
 * velocity model's node velocity over the current and the previous step), in m/s, as [3][N]
 * float64 in host memory (solid voxels 0; the third component is 0 in 2D).  E_STATE without
 * advection. */
int lbm_ms_get_velocity(lbm_ms_t h, double* u_host);

/* Post-collision populations of the current state, decoded to float64, host [2][Q][N], in the
 * velocity order of lbm_ms_lattice_info. */
int lbm_ms_get_populations(lbm_ms_t h, double* f_host);

/* Species inventory sum_r X_s (fluid nodes) of the current state, and the amounts that the next
 * step moves in through the inlet face and out through the outlet face (species 1 and 2). */
int lbm_ms_mass_balance(lbm_ms_t h, double inventory[2], double inflow[2], double outflow[2]);

/* Checkpoint: *bytes = size when host_buf is NULL; otherwise writes the state (populations,
 * node shift field, residual snapshot, step count, parameter hash) into host_buf. */
int lbm_ms_save_state(lbm_ms_t h, void* host_buf, size_t* bytes);
int lbm_ms_load_state(lbm_ms_t h, const void* host_buf, size_t bytes);

int lbm_ms_get_info(lbm_ms_t h, lbm_ms_info* info);

/* Velocity set of a lattice: *q, e[3*q] (ex, ey, ez), w[q] (either pointer may be NULL). */
int lbm_ms_lattice_info(int lattice, int* q, int* e, double* w);

/* The 2D step's work list for a host mask (nx*ny bytes, 1 = solid, used as given), host only:
 * the tiles that lbm_ms_set_geometry would build for launch shape (tile_y, rows) of
 * lbm_ms_tile_options.  *n_tiles and *n_ent receive the counts; with tiles and ent non-NULL
 * (8 int32 per tile, n_ent uint32) the lists are copied out too, so call once for the counts and
 * again with buffers of that size.  Per tile: x0, y0, instance (0), 0, then the offset and count
 * of its own entries and of its halo entries in ent.  An entry packs the node's moment-tile
 * coordinates as cy << 8 | cx, (x, y) = (x0 + cx - 1, y0 + cy - 1), with y taken periodically.
 * E_ARG for a 3D lattice or a shape that is not compiled. */
int lbm_ms_work_list(int lattice, int nx, int ny, const uint8_t* solid, int tile_y, int rows,
                     int64_t* n_tiles, int64_t* n_ent, int32_t* tiles, uint32_t* ent);

/* Launch shapes compiled for a lattice and storage mode (precision, shift_mode): writes up to cap
 * (tile_y, chunk_z) pairs, returns the count (at most 16).  3D: 64 x tile_y columns marching
 * chunk_z planes; tile_y 4 and 8 give each lane one voxel of a 64 x tile_y plane, tile_y 12 and 16
 * (global-shift storage in FP32, FP16 or BF16 only) give the 512 lanes of a workgroup the fluid
 * voxels of a 64 x tile_y plane in order, from per-(column, plane) lists that the handle builds at
 * lbm_ms_set_geometry and lbm_ms_set_tile (2 bytes per fluid node).  2D: workgroups of 32 tile_y
 * lanes, one fluid node per lane; chunk_z = 0 for fixed 64 x tile_y tiles (a denser tile is split
 * into parts), chunk_z > 0 for packed tiles that grow row by row in each 64-wide strip up to
 * chunk_z rows or 32 tile_y fluid nodes. */
int lbm_ms_tile_options(int lattice, int precision, int shift_mode, int* tile_y, int* chunk_z,
                        int cap);

/* Change the launch shape of an existing handle (one of lbm_ms_tile_options). */
int lbm_ms_set_tile(lbm_ms_t h, int tile_y, int chunk_z);

/* ---------------------------------------------------------------------------------------------
 * Batched solves (D2Q9 or D2Q5): many independent porous slices of uneven size, each with its own
 * geometry, inlet composition and current density, advanced together.  Every step is one kernel
 * launch over the combined tile work list of all still-active instances; a converge call captures
 * check_every steps into a hipGraph on the batch's own stream and replays it, checks every
 * instance's residual, and retires converged instances from the work list.  One point of a
 * polarization curve (Eq. 43 at each current density) per instance.
 * ------------------------------------------------------------------------------------------- */
typedef struct lbm_ms_batch_s* lbm_ms_batch_t;

typedef struct {
    int nx, ny;                /* nodes of this instance (nz = 1) */
    const uint8_t* solid;      /* host mask nx*ny, 1 = solid (cleaned as in lbm_ms_set_geometry) */
    double X_in[3];            /* inlet mole fractions (Eq. 36) */
    double j_A_per_m2;         /* current density (Eq. 39) */
} lbm_ms_instance_desc;

/* Device bytes for count instances with the shared parameters common (its lattice must be
 * LBM_MS_D2Q9; nx, ny, nz are taken from each descriptor).  0 if invalid. */
size_t lbm_ms_batch_workspace_bytes(const lbm_ms_params* common, const lbm_ms_instance_desc* inst,
                                    int count);

/* Create the batch: geometry clean-up, index maps, work lists and boundary data of every
 * instance.  On failure *out is NULL and lbm_ms_batch_last_error(NULL) tells why on this thread;
 * E_GEOM names the first instance whose outlet is unreachable.
 * The caller owns d_workspace; the batch owns a stream of its own, ordered after common.stream
 * at every call and before it on return. */
int lbm_ms_batch_create(const lbm_ms_params* common, const lbm_ms_instance_desc* inst, int count,
                        void* d_workspace, size_t bytes, lbm_ms_batch_t* out);

/* Initial state of every instance: uniform inlet composition (X0 == NULL) or a concatenation of
 * per-instance [3][nx*ny] float64 fields, host (on_device = 0) or device memory.  Re-activates
 * every instance. */
int lbm_ms_batch_init(lbm_ms_batch_t b, const double* X0, int on_device);

/* nsteps steps of every active instance (one launch per step; asynchronous). */
int lbm_ms_batch_step(lbm_ms_batch_t b, int64_t nsteps);

/* nsteps eager steps bracketed by HIP events on the batch's launch stream; *ms = elapsed
 * milliseconds (synchronizes). */
int lbm_ms_batch_time_steps(lbm_ms_batch_t b, int64_t nsteps, double* ms);

/* Steps in hipGraph-captured chunks of check_every until every instance's residual (as
 * lbm_ms_residual, bit for bit; the checks of all instances run as one reduction over the batch
 * with one read-back) is below tol or max_steps is reached.  An instance whose check fails
 * (E_NEG_FRACTION when its current exceeds what its pores can supply, E_DIVERGED, E_TAU_CLAMP)
 * retires with that status while the others go on.  Per instance (each pointer may be NULL):
 * steps_taken[k], residual[k], status[k] (0 = converged, E_NOT_CONVERGED, or the failure).
 * Retired instances stay out of the work list (and report their retirement status, 0 steps and
 * residual +inf in later calls) until lbm_ms_batch_init.
 * Returns 0 if every instance converged, else the first nonzero status in instance order. */
int lbm_ms_batch_converge(lbm_ms_batch_t b, double tol, int64_t max_steps, int check_every,
                          int64_t* steps_taken, double* residual, int* status);

/* Per-instance overpotential (Eq. 43) into eta[count]. */
int lbm_ms_batch_overpotential(lbm_ms_batch_t b, double* eta);

/* The single-instance handle of instance k (for lbm_ms_get_fields, lbm_ms_residual, ...).  It
 * stays owned by the batch; do not destroy it or step it on its own while the batch runs. */
lbm_ms_t lbm_ms_batch_instance(lbm_ms_batch_t b, int k);

/* Active instances, total fluid nodes of the active instances, and active tiles. */
int lbm_ms_batch_stats(lbm_ms_batch_t b, int* active, int64_t* fluid_nodes, int* tiles);

/* Launch shape of every instance: one (tile_y, rows) pair of lbm_ms_tile_options for the batch's
 * lattice (rows = 0: fixed 64 x tile_y tiles, else packed tiles of at most rows rows). */
int lbm_ms_batch_set_tile(lbm_ms_batch_t b, int tile_y, int rows);

/* Use (1) or bypass (0) hipGraph capture in lbm_ms_batch_converge (default 1). */
int lbm_ms_batch_use_graphs(lbm_ms_batch_t b, int enable);

const char* lbm_ms_batch_last_error(lbm_ms_batch_t b);
void lbm_ms_batch_destroy(lbm_ms_batch_t b);

/* The last error of handle h; with h == NULL, why the last lbm_ms_create, lbm_ms_batch_create or
 * lbm_ms_workspace_bytes (returning 0) that failed on the calling thread failed. */
const char* lbm_ms_last_error(lbm_ms_t h);
const char* lbm_ms_status_string(int status);

/* Release host resources; never frees the caller's workspace.  Synchronizes the stream. */
void lbm_ms_destroy(lbm_ms_t h);

#ifdef __cplusplus
}
#endif

#endif /* LBM_MS_H */
