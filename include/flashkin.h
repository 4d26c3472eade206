/*
 * flashkin.h -- C-ABI of the MI355X (gfx950) library that advances the
 * 1D2V electron distribution of the vacuum surface-flashover model of
 * Sun et al., "An alternative simulation approach for surface flashover in
 * vacuum using a 1D2V continuum and kinetic model" (arXiv 2303.14119).
 *
 * One step (Section 2) advances f(x, v_x, v_y) on a cell-centred phase-space
 * grid by explicit first-order upwind transport (the paragraph after Eq 2):
 * x by v_x, then v_x by a_x = -e E_x(x)/m, then v_y by a_y = -e E_y/m, then
 * the field-emission band source (Eq 7).  At the dielectric (x = 0) the
 * primary flux (Eq 13-14) is absorbed, secondaries are re-emitted through
 * the SEE yield matrix (Eq 8-12) with the half-Maxwellian of Eq 15-16, and
 * the surface charge is updated by Eq 18.  Everything reaching x = L is
 * absorbed (Eq 17).  E_x comes from the 1D Gauss law with
 * E_x(0) = sigma / 2 eps0 (the paragraph on the velocity advections).
 *
 * Conventions for every call:
 *   - Return value: FK_OK (0) or a negative FK_E_* code.  No C++ exception
 *     crosses this boundary.  fk_last_error() gives a message.
 *   - Device pointers are HIP device addresses on the current device; host
 *     pointers are ordinary process memory.  Nothing passed in is freed by
 *     the library unless the call says so.
 *   - A context is not thread-safe: one host thread at a time per context.
 *   - Work is queued on the HIP stream given at creation (NULL = the null
 *     stream).  Calls that return data to the host synchronise that stream.
 *   - f is laid out [k][i][j] (x index k slowest, v_y index j fastest),
 *     dense, element type FK_F32 (float) or FK_F64 (double).
 *   - Units are SI; energies and temperatures named *_ev are in eV.
 */
#ifndef FLASHKIN_H
#define FLASHKIN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FK_ABI_VERSION 5u   /* 2: fk_batch_info_t gained single_threads; 3: fk_params gained t_e_ev, ln_lambda; 4: r_refl;
                              5: r_inel, scheme */

/* element type of f */
enum { FK_F32 = 0, FK_F64 = 1 };

/* normalisation of the emission row (Eq 15-16) */
enum {
    FK_EMIT_DISCRETE = 0, /* scaled so the emitted flux on the grid equals Gamma_see */
    FK_EMIT_ANALYTIC = 1  /* the continuum prefactor of Eq 15 */
};

/* parts of the step (all on = FK_PHYS_ALL); tests switch parts off */
enum {
    FK_PHYS_X = 1,           /* x advection with the wall and vacuum boundaries */
    FK_PHYS_VX = 2,          /* v_x advection by -e E_x / m */
    FK_PHYS_VY = 4,          /* v_y advection by -e E_y / m */
    FK_PHYS_SRC = 8,         /* band source (Eq 7) */
    FK_PHYS_SEE = 16,        /* secondary emission (Eq 8-16) */
    FK_PHYS_SELF_FIELD = 32, /* E_x from sigma and the electron space charge */
    FK_PHYS_ALL = 63,
    /* Electron-electron collisions, the BGK term of Eq 3-5: each cell relaxes
     * towards n_e(x) times the Maxwellian of Eq 5 at t_e_ev, at the frequency
     * nu_ee(n_e) of Eq 4 with ln_lambda.  Opt-in (not part of FK_PHYS_ALL).
     * Taken explicitly on f^n and n^n and added to the swept f; the
     * Maxwellian is normalised on the grid, so the term moves no electrons
     * between x planes. */
    FK_PHYS_BGK = 64,
    /* With FK_PHYS_SELF_FIELD: E_x = sigma / 2 eps0 (+ ex_external) at every
     * x, the electrons' own space charge left out.  This is the field of the
     * single-particle theory of Eq 19-20 (Section 3); it separates the space
     * charge's share of the saturated sigma.  Opt-in. */
    FK_PHYS_NO_SPACE_CHARGE = 128
};

/* advection scheme (fk_params.scheme) */
enum {
    FK_SCHEME_UPWIND = 0,   /* the paper's explicit first-order upwind step (Section 2, after Eq 2), split
                             * x, v_x, v_y, source */
    FK_SCHEME_LIMITED2 = 1  /* an accuracy extension beyond the paper for coarse grids: each 1D sweep in flux
                             * form with a minmod-limited slope (the face carries the upwind cell's value
                             * moved towards the face by (1 - |c|)/2 times its slope; slopes are zero in
                             * the first and last cell of every line, so every boundary face carries the
                             * upwind value as in scheme 0), and the split order reversed on odd steps
                             * (source, v_y, v_x, x) so that two steps form a symmetric composition.  On
                             * a reversed step the electrons absorbed at the wall and at x = L are those
                             * of the array the x sweep transports; the yield, emission row and
                             * reflection still come from f^n.  FK_F32 or FK_F64; not with FK_PHYS_BGK or
                             * in a batch (FK_E_INVALID).  Tiles of 4 or 8 v_x rows; nvy up to 768 (FK_F32)
                             * or 384 (FK_F64) with 4 rows, 512 or 256 with 8 */
};

/* error codes */
enum {
    FK_OK = 0,
    FK_E_INVALID = -1,   /* bad argument or parameter */
    FK_E_OOM = -2,       /* device or host allocation failed */
    FK_E_HIP = -3,       /* a HIP runtime call failed */
    FK_E_CFL = -4,       /* a Courant number, or nu_ee dt with FK_PHYS_BGK, exceeded one (sticky until fk_write_state) */
    FK_E_NONFINITE = -5, /* a moment or flux became NaN/Inf (sticky until fk_write_state) */
    FK_E_STATE = -6      /* call not valid in the object's current state */
};

/* Parameters of one run.  Set struct_size = sizeof(fk_params) and
 * abi_version = FK_ABI_VERSION.  Inputs of Section 2's parameter list. */
typedef struct {
    uint32_t struct_size, abi_version;
    int32_t nx, nvx, nvy;    /* cells in x (normal to the surface), v_x, v_y; each >= 1; nvy <= 1024 for
                              * FK_F32 and <= 960 for FK_F64 (a tile's v_y exchange must fit in 64 KB of
                              * LDS; larger values fail with FK_E_INVALID) */
    int32_t dtype;           /* FK_F32 or FK_F64 */
    double length_m;         /* domain extent normal to the surface (x in [0, L]) */
    double vmax_x, vmax_y;   /* velocity box [-vmax, vmax] in each direction, m/s */
    double dt;               /* time step, s; 0 selects cfl * min(dx/vmax_x, dv_x/|a_y|, dv_y/|a_y|) */
    double cfl;              /* CFL fraction used when dt = 0 */
    double ey;               /* applied tangential field E_y, V/m (negative: cathode on the left) */
    double delta_max;        /* SEY maximum (Eq 8) */
    double a_max_ev;         /* normal-incidence energy of the SEY maximum (Eq 9) */
    double ks;               /* surface smoothness factor k_s (Eq 8-9), 1 for a normal surface */
    double t_se_ev;          /* secondary emission temperature T_se (Eq 15) */
    double j_src;            /* seed current density of the band source, A/m^2 (Eq 7) */
    double x_src_lo, x_src_hi; /* source band in x, m (the paper: 10-15 um) */
    double t_src_ev;         /* temperature of the source VDF (Eq 7) */
    int32_t emission_norm;   /* FK_EMIT_DISCRETE or FK_EMIT_ANALYTIC */
    uint32_t physics_mask;   /* FK_PHYS_* bits */
    double ex_external;      /* uniform E_x added to the self field, V/m */
    int32_t trace_stride;    /* record observables every trace_stride steps (>= 1) */
    int32_t trace_cap;       /* records held on the device between drains (>= 1) */
    int32_t tile_rows;       /* v_x rows per tile: 4, 8, 12 or 16 (12: FK_F32, nvy <= 512; 16: FK_F32, nvy <= 448;
                              * 8: nvy <= 960 in FK_F32, 448 in FK_F64), 0 = library choice */
    int32_t tile_planes;     /* x planes per tile; 0: chosen at creation from the sweep kernel's occupancy: the longest run (16..128) that keeps 8 waves resident per compute unit, or all a unit holds, with the workgroups spread evenly (fk_validate reports a host-side estimate, fk_query the choice); batch instances get 16 */
    double t_e_ev;           /* FK_PHYS_BGK: temperature of the collisional equilibrium (Eq 4-5), eV, > 0 */
    double ln_lambda;        /* FK_PHYS_BGK: Coulomb logarithm of Eq 4 (the paper: 10), > 0 */
    double r_refl;           /* elastic share of the wall reflection coefficient R_f (Section 2, after
                              * Eq 14), in [0, 1]: a fraction r_refl of the electrons reaching the dielectric
                              * returns specularly (v_x -> -v_x) through the emission row.  0: none */
    double r_inel;           /* inelastic share of R_f, in [0, 1 - r_refl]: a fraction r_inel of the arrivals
                              * has given its energy to the wall and leaves with the secondaries' Eq 15
                              * half-Maxwellian at t_se_ev (the emission row carries Gamma_see + r_inel
                              * Gamma_pe in that shape).  1 - r_refl - r_inel of the arrivals induce SEE
                              * (Gamma_see scales by it), and reflected electrons of either share deposit no
                              * charge in Eq 18.  0: none */
    int32_t scheme;          /* FK_SCHEME_UPWIND or FK_SCHEME_LIMITED2 */
    int32_t reserved0;       /* 0 */
} fk_params;

/* Observables of the state (f^n, sigma^n) after n steps.  The fluxes are
 * those of f^n, i.e. the ones step n+1 will use. */
typedef struct {
    int64_t step;            /* n */
    double t;                /* n dt, s */
    double sigma;            /* surface charge sigma^n, C/m^2 (Eq 18) */
    double sigma_lo;         /* compensation term of the sigma sum (sigma + sigma_lo is the value) */
    double g_pe;             /* primary flux into the wall, 1/(m^2 s) (Eq 13-14) */
    double g_see;            /* secondary flux (Eq 12, 14), times 1 - r_refl - r_inel */
    double g_top;            /* flux leaving through x = L */
    double emitted;          /* flux carried by the emission row, sum v_x f_ghost dv_x dv_y (secondaries plus both reflected shares) */
    double loss_v;           /* electrons/m^2 lost through the velocity-box edges in step n */
    double n_total;          /* electrons/m^2 in the domain */
    double resid;            /* particle balance residual of step n, electrons/m^2 */
} fk_state;

/* Derived quantities of a parameter set. */
typedef struct {
    double dx, dvx, dvy, dt;
    double courant_x;        /* max |v_x| dt / dx over the grid */
    double courant_vy;       /* |a_y| dt / dv_y */
    int64_t cells;           /* nx * nvx * nvy */
    int32_t tile_rows, tile_planes, block, n_tiles;
    uint64_t bytes_device;   /* device memory the context allocates */
} fk_info;

typedef struct fk_ctx fk_ctx;
typedef struct fk_batch fk_batch;

/* Error text for a code; and the last message of a context (NULL: of the
 * calling thread's last failed create). */
const char* fk_error_string(int code);
const char* fk_last_error(const fk_ctx* ctx);

/* Validate a parameter set and derive grid spacings, time step and launch
 * shape.  Host only; does not touch the GPU.  out may be NULL. */
int fk_validate(const fk_params* p, fk_info* out);

/* Create a context: builds the grids and the tables of Eq 7, 8-11 and 15 on
 * the device, sets f = 0, sigma = 0, step 0.  stream is a hipStream_t (or
 * NULL).  The context owns its device memory. */
int fk_create(const fk_params* p, void* stream, fk_ctx** out);

/* As fk_create, but f lives in two caller-owned device buffers of
 * nx*nvx*nvy elements each (ping-pong).  The caller keeps them alive and
 * does not touch them until fk_destroy. */
int fk_create_borrowed(const fk_params* p, void* stream, void* f_a, void* f_b, fk_ctx** out);

int fk_destroy(fk_ctx* ctx);

/* Derived quantities of the context's parameters. */
int fk_query(const fk_ctx* ctx, fk_info* out);

/* Queue nsteps >= 0 steps on the stream (asynchronous).  Returns a sticky
 * error seen by an earlier fk_sync. */
int fk_step(fk_ctx* ctx, int64_t nsteps);

/* Wait for queued work; returns FK_E_CFL or FK_E_NONFINITE if a step raised
 * one since the last fk_write_state. */
int fk_sync(fk_ctx* ctx);

/* Copy the current f (layout and type as above) to dst, which holds
 * dst_bytes >= nx*nvx*nvy*sizeof(element) bytes; on the device if
 * dst_on_device != 0, else in host memory. */
int fk_read_f(fk_ctx* ctx, void* dst, size_t dst_bytes, int dst_on_device);

/* Observables of the current state (synchronises). */
int fk_read_state(fk_ctx* ctx, fk_state* out);

/* E_x at the nx cell centres (V/m) and n_e (1/m^3) of the current state;
 * either pointer may be NULL.  Host memory unless dst_on_device != 0.
 * The x-resolved enclosed charge is 2 eps0 E_x. */
int fk_read_field(fk_ctx* ctx, double* ex, double* ne, int dst_on_device);

/* Host copies of the FP64 tables: delta (Eq 8-11, 0 where v_x >= 0), the
 * emission shape exp(-m v^2 / 2 T_se) (0 where v_x <= 0), the normalised
 * source VDF (nvx*nvy each, [i][j]) and the band weights (nx).  Any pointer
 * may be NULL. */
int fk_read_tables(fk_ctx* ctx, double* delta, double* ghat, double* fsrc, double* wband);

/* Drain the trace ring: copies up to cap records made since the last drain
 * (oldest first) to dst (host), count in *n_out.  If more than trace_cap
 * records were made since the last drain, only the newest trace_cap remain
 * and the call returns FK_E_STATE after copying them. */
int fk_read_trace(fk_ctx* ctx, fk_state* dst, size_t cap, size_t* n_out);

/* Replace the state: f (NULL keeps the current f; device memory if
 * src_on_device, else host), sigma = sigma + sigma_lo, and the step counter.
 * Clears sticky errors and the trace history.  Used for warm starts,
 * checkpoint restore and tests. */
int fk_write_state(fk_ctx* ctx, const void* f, int src_on_device, double sigma, double sigma_lo,
                   int64_t step);

/* The x-resolved enclosed charge of the current state,
 * sigma_enc(x) = sigma - 2 e int_0^x n_e(x') dx' with n_e constant over each
 * cell (2 eps0 times the self field of the Section 2 field solve; equal to
 * sigma at the dielectric), at npts >= 2 uniform points x_p = p L / (npts - 1);
 * into out (host, or device if dst_on_device).  FK_E_INVALID for npts < 2. */
int fk_read_profile(fk_ctx* ctx, int npts, double* out, int dst_on_device);

/* Warm start from a predicted profile (npts >= 2 values of sigma_enc at the
 * uniform points above; host or device memory): sigma = profile[0] and
 * f(x_k, v) = n_k M(v), where n_k = (S(k dx) - S((k+1) dx)) / (2 e dx) is the
 * cell-averaged electron density whose enclosed charge is the piecewise-
 * linear profile S (clamped at zero) and M the Maxwellian at t_ev normalised
 * on the velocity grid.  The step counter is set to step; otherwise as
 * fk_write_state. */
int fk_warm_start(fk_ctx* ctx, const double* profile, int npts, int src_on_device, double t_ev, int64_t step);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the work of
 * fk_create_borrowed + fk_write_state + fk_step(nsteps) + fk_read_state in
 * one call that allocates nothing.  f_a and f_b are the caller's two device
 * buffers of nx*nvx*nvy elements (type of p->dtype); f_a holds f^0 on entry
 * and both are overwritten; after the call the state is in f_a if nsteps is
 * even, in f_b if odd.  sigma + sigma_lo and step give the starting surface
 * charge and step counter.  state_out (device memory, may be NULL) receives
 * the observables of the final state as fk_read_state gives them, and
 * flags_out (device, may be NULL) its flags: bit 0 a Courant number above
 * one, bit 1 a non-finite moment (what fk_sync turns into FK_E_CFL /
 * FK_E_NONFINITE).  The work is queued on stream and the call returns
 * without waiting; results are the same, bit for bit, as with a context.
 * Tables, tile partials, the small state and the trace ring (trace_cap
 * records; they are not read back) live in a file-scope array of 32 MiB per
 * GPU that the library holds until the process ends; parameters needing more
 * (in practice nx * ceil(nvx/4) * 8 bytes of partials plus 32 bytes per
 * velocity cell of tables) fail with FK_E_INVALID.  Every call on a GPU
 * shares that array and the call clears what it uses first: calls that
 * overlap on one GPU (other streams or threads) race and give wrong results.
 * Errors: FK_E_INVALID for bad arguments or parameters, FK_E_HIP for a failed
 * launch; fk_last_error(NULL) gives the message. */
int fk_step_noalloc(const fk_params* p, void* stream, void* f_a, void* f_b, double sigma, double sigma_lo,
                    int64_t step, int64_t nsteps, fk_state* state_out, uint32_t* flags_out);

/* Saturation test of Section 2 (sigma, Gamma_pe and Gamma_see each change
 * by at most rtol relative within a window of window_s seconds), applied to
 * the trace history drained so far (the call drains the ring first).
 * *out = 1 if saturated, 0 if not or if the history is shorter than the
 * window. */
int fk_saturated(fk_ctx* ctx, double window_s, double rtol, int* out);

/* The same test on a caller-held trace (host only, no GPU). */
int fk_saturation_check(const fk_state* trace, size_t n, double window_s, double rtol, int* out);

/* Field-emission current density at the cathode triple junction, Eq 6
 * (Fowler-Nordheim), with the work function e*phi_m = phi_ev electron-volts
 * and the junction field E = beta * |e_field| (Section 2 takes E_CTJ = |E_y|,
 * i.e. beta = 1; beta > 1 stands for a local field enhancement).  Host only.
 * *j_out in A/m^2, the rate j_src of the Eq 7 band source; 0 where the
 * exponential underflows (|E_y| of a few MV/m with beta = 1).
 * FK_E_INVALID for phi_ev <= 0, beta <= 0, a non-finite field or NULL out. */
int fk_fn_current(double e_field, double phi_ev, double beta, double* j_out);

/* Surface charge along the insulator from the trace of one 1D element (a
 * reading of Section 4's comparison, where the 2D charging time is the
 * insulator length over the avalanche speed v_seea): the avalanche front
 * leaves the junction (y = 0) at t = 0 and moves at v_seea, and an element
 * at y charges as the 1D run did from the moment the front reached it:
 *   sigma(y, t) = sigma_1D(t - y / v_seea),
 * linear between trace records (sigma + sigma_lo) and from 0 at the front
 * to the first record (the run starts uncharged, Section 2), 0 ahead of
 * the front (y > v_seea t) and the last record's value past the trace.
 * Host only.  trace: n >= 1 records in increasing t; y: ny positions (m);
 * out: ny values (C/m^2).  FK_E_INVALID for v_seea <= 0, NULL arrays with
 * n or ny > 0, or records out of order. */
int fk_sigma_along(const fk_state* trace, size_t n, double v_seea, double t, const double* y, size_t ny,
                   double* out);

/* Kernel timing.  fk_set_profiling(ctx, every) with every >= 1 switches
 * profiling on: fk_step then launches every step directly (no graphs) and,
 * for every `every`-th step counted from the call (the first included),
 * records three HIP events on the context's stream: before and after the
 * sweep launch and after the reduction and field kernels.  every = 0
 * switches it off; every < 0 is FK_E_INVALID.  Each call drops the events
 * taken so far.  fk_kernel_times synchronises and returns the summed
 * milliseconds and counts of the sampled sweep launches and of their
 * reduction-and-field intervals. */
int fk_set_profiling(fk_ctx* ctx, int every);
int fk_kernel_times(fk_ctx* ctx, double* sweep_ms, int64_t* sweep_count, double* field_ms,
                    int64_t* field_count);

/* Tiling autotuner (a project addition; the paper prescribes no kernel
 * layout).  Times trial_steps >= 2 steps for each candidate tiling (v_x rows
 * 4/8/12/16 x x planes 16/32/64/128 that fit) and keeps the fastest.  The state
 * (f, sigma, step, trace history) is the same afterwards.  The chosen layout
 * is written to *chosen if it is not NULL. */
int fk_autotune(fk_ctx* ctx, int trial_steps, fk_info* chosen);

/* ---- batched instances ---------------------------------------------------
 * n independent runs of uneven sizes (the parameter sweep that feeds the
 * surrogate) advanced together; a project addition beyond the paper, whose
 * runs each follow Section 2.  Persistent sweep launches take (instance,
 * x chunk, v_x tiles) work items largest first from an atomic counter; one
 * field launch then reduces and solves every instance (a workgroup each);
 * steps are replayed from HIP graphs.  Every instance is FK_F32 with
 * nvy <= 256 and starts at f = 0, sigma = 0.  If any member has
 * FK_PHYS_BGK the batch runs the sweep variant with the collision term
 * (members without it skip the term).
 *   mode 0: split launches: up to four sweep launches per step, by tile
 *           body and workgroup width;
 *   mode 1: autotune: time short trial runs of tilings, grid sizes, item
 *           schedules and both launch modes (mode 2 at 256 and at 192
 *           threads per workgroup), keep the fastest, then reset the
 *           instances to f = 0;
 *   mode 2: one sweep launch per step for all instances and tiles, in
 *           workgroups of 256 threads (on 64 uneven instances the faster
 *           of the untuned modes);
 *   mode 3: as mode 2 with workgroups of 192 threads (no idle wave beside
 *           a 192-lane v_y block), or 256 if an instance has nvy > 192.
 * Results are bitwise the same in every mode and equal to single contexts
 * with the same tiling. */
typedef struct {
    int32_t n;             /* instances */
    int32_t tile_rows;     /* v_x rows per tile */
    int32_t tile_planes;   /* x planes per tile of instance 0 */
    int32_t grid;          /* workgroups of the largest persistent sweep launch */
    int32_t items;         /* work items per step */
    int64_t lds_bytes;     /* LDS per workgroup */
    int64_t cells;         /* sum of nx * nvx * nvy over the instances */
    int32_t schedule;      /* 0: items from an atomic counter, 1: static round-robin */
    int32_t sweep_launches;/* sweep launches per step (1 in mode 2) */
    int32_t single_threads;/* threads per workgroup of the single sweep launch (256, or 192 if the autotuner chose it); 0 with split launches */
} fk_batch_info_t;

int fk_batch_create(const fk_params* params, int n, void* stream, int mode, fk_batch** out);
int fk_batch_destroy(fk_batch* batch);

/* Queue nsteps steps of every instance (asynchronous). */
int fk_batch_step(fk_batch* batch, int64_t nsteps);

/* Wait; returns the first error (CFL, non-finite) among the active
 * instances and its index in *first_bad (-1 if none; may be NULL).  After an
 * error fk_batch_step refuses to run until the flagged instances are retired;
 * the others are unaffected (instances share no data). */
int fk_batch_sync(fk_batch* batch, int* first_bad);

/* Non-owning view of instance i, valid until fk_batch_destroy: the fk_read_*,
 * fk_write_state, fk_saturated and fk_query calls work on it; fk_step on a
 * view returns FK_E_STATE. */
int fk_batch_get(fk_batch* batch, int i, fk_ctx** view);

int fk_batch_info(const fk_batch* batch, fk_batch_info_t* out);

/* Stop stepping instances idx[0..n-1] (e.g. saturated or flagged ones);
 * their state stays readable through the views.  Clears the batch's pending
 * error and rebuilds the work list and graphs. */
int fk_batch_retire(fk_batch* batch, const int* idx, int n);
const char* fk_batch_last_error(const fk_batch* batch);

/* ---- surrogate network ---------------------------------------------------
 * A multilayer perceptron (GELU hidden layers, linear output) that maps the
 * run parameters to the saturated state; a project addition beyond the
 * paper.  Trained on the GPU: BF16 MFMA GEMMs with FP32 accumulation, FP32
 * master weights, MSE loss, AdamW.  The library owns the network's device
 * memory; inputs and targets are FP32 device arrays given by the caller.
 * Parameters are exchanged as one flat FP32 vector
 * [W_1 (dims[1] x dims[0], row-major), b_1, W_2, b_2, ...]. */
typedef struct fk_mlp fk_mlp;

/* n_layers weight layers, widths dims[0..n_layers]; max_batch a multiple of
 * 16.  Parameters start at zero (set them with fk_mlp_set_params). */
int fk_mlp_create(int n_layers, const int32_t* dims, int max_batch, void* stream, fk_mlp** out);
int fk_mlp_destroy(fk_mlp* net);
const char* fk_mlp_last_error(const fk_mlp* net);
int fk_mlp_num_params(const fk_mlp* net, int64_t* count);
int fk_mlp_set_params(fk_mlp* net, const float* src, int src_on_device);
int fk_mlp_get_params(fk_mlp* net, float* dst, int dst_on_device);
/* Gradients of the last fk_mlp_backward, same flat layout. */
int fk_mlp_get_grads(fk_mlp* net, float* dst, int dst_on_device);

/* x: device FP32 [M][dims[0]]; y (device FP32 [M][dims[n_layers]], may be
 * NULL).  Keeps the activations for a following fk_mlp_backward. */
int fk_mlp_forward(fk_mlp* net, const float* x, int M, float* y);

/* Mean-squared-error loss against target (device FP32 [M][dims[n_layers]])
 * for the batch of the last forward (M a multiple of 16); computes every
 * parameter gradient.  *loss (host, may be NULL) receives the loss, which
 * synchronises the stream; with NULL the call only queues work.  Either
 * way the loss is added to a device-side running sum (fk_mlp_take_loss). */
int fk_mlp_backward(fk_mlp* net, const float* target, int M, float* loss);

/* Synchronises; *mean (may be NULL) receives the mean of the losses of the
 * fk_mlp_backward calls since the last take (0 if none) and *count (may be
 * NULL) their number; the running sum starts again from zero. */
int fk_mlp_take_loss(fk_mlp* net, double* mean, int64_t* count);

/* One AdamW step (decoupled weight decay on the weights, none on biases)
 * with bias-corrected moments; step counts from 1. */
int fk_mlp_adamw(fk_mlp* net, double lr, double beta1, double beta2, double eps, double weight_decay,
                 int64_t step);

/* One whole training step on a batch: the forward pass, the loss against
 * target, every gradient and the AdamW step, as fk_mlp_forward,
 * fk_mlp_backward (loss not read back) and fk_mlp_adamw would do it, with
 * fewer launches: the first layer's GEMM reads the FP32 features itself,
 * the loss and its gradient come out of the output layer's
 * GEMM, and one launch forms every weight gradient and applies AdamW to it
 * tile by tile, updates the biases and adds up the loss.  x: device FP32
 * [M][dims[0]]; target: device FP32 [M][dims[n_layers]]; M a multiple of 16
 * up to max_batch.  The loss joins the running sum of fk_mlp_take_loss and
 * the gradients stay readable with fk_mlp_get_grads.  Same results as the
 * three calls up to summation order. */
int fk_mlp_train_step(fk_mlp* net, const float* x, const float* target, int M, double lr, double beta1,
                      double beta2, double eps, double weight_decay, int64_t step);
int fk_mlp_sync(fk_mlp* net);

#ifdef __cplusplus
}
#endif

#endif /* FLASHKIN_H */
