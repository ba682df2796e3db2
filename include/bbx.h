/*
 * bbx.h -- C ABI of the MI355X monodomain step library (libbbx.so).
 *
 * The library advances the monodomain reaction-diffusion system of the paper
 * (Antonioletti et al., "BeatBox", arXiv:1605.06015, eq (monodomain)) on a
 * regular Cartesian grid with void points, by the explicit scheme of the
 * sections "Splitting the problem into parts" and "Kinetics solvers": the
 * anisotropic no-flux diffusion stencil ("Monodomain diffusion and boundary
 * conditions", eqs (Lu), (nonflux), (sigma) and the weight formulas), fused
 * with the per-voxel ionic update (forward Euler, eq (Euler); Rush-Larsen for
 * gates, eqs (RL), (RLcoeff)) and a stimulus current.  All compute runs in
 * HIP kernels for gfx950.
 *
 * Conventions (all entry points):
 *   - Grid layout: box index idx = x + nx*(y + ny*z), x fastest.  Host arrays
 *     over the box have nx*ny*nz entries (times 3 for fibres).
 *   - Units: V in mV, t in ms, D in mm^2/ms, h in mm, currents in pA/pF
 *     (= mV/ms with the membrane capacitance normalised).  Barkley, ZFK and
 *     FHN are dimensionless.
 *   - Ownership: every host input array is copied before the call returns;
 *     the caller keeps it.  The library owns all device memory it allocates
 *     and frees it in bbx_grid_destroy.  Device output pointers passed to
 *     bbx_readout stay owned by the caller and must remain valid until the
 *     grid's stream has passed the copy.
 *   - Errors: every call returns BBX_OK or a negative code and leaves the grid
 *     unchanged on error; bbx_last_error() returns the message of the calling
 *     thread's last failure.  Argument validation happens before any device
 *     work.  No C++ exception crosses the ABI.
 *   - Streams: work is enqueued on the stream given at creation (NULL = the
 *     null stream).  bbx_step is asynchronous except for its optional
 *     finite-value check (bbx_nan_check_set).
 *   - Threading: a grid is not thread-safe; distinct grids are independent.
 *   - Log: with the environment variable BBX_LOG set to a non-zero value (read
 *     once, at the library's first log), every failed call writes its code and
 *     message, and grid creation, model set-up and surrogate attachment write
 *     one line each, to stderr, prefixed "bbx: ".
 */
#ifndef BBX_H
#define BBX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bbx_grid bbx_grid;

/* Return codes. */
enum {
    BBX_OK = 0,
    BBX_EINVAL = -1,     /* bad argument (null pointer, size, count, non-normalisable fibre) */
    BBX_ENOMEM = -2,     /* device allocation failed */
    BBX_EDEVICE = -3,    /* a HIP call failed */
    BBX_ESTATE = -4,     /* call out of order (e.g. bbx_step before bbx_model_set) */
    BBX_EUNSTABLE = -5,  /* dt above the explicit-diffusion stability bound */
    BBX_ENUMERIC = -6,   /* a non-finite state value was found */
    BBX_ENOTSUP = -7     /* combination not supported */
};

/* Arithmetic precision of state, stencil and kinetics. */
enum { BBX_FP32 = 0, BBX_FP64 = 1 };

/* Coupling of diffusion and kinetics ("Splitting the problem into parts"):
 *  ADDITIVE: V+ = V + dt(-I_ion(V,g) + I_stim + LV), kinetics at (V, g)
 *            (the "intermediate expression" scheme);
 *  SPLIT:    V* = V + dt LV, then V+ = V* + dt(-I_ion(V*,g) + I_stim),
 *            kinetics at (V*, g) (Lie operator splitting). */
enum { BBX_SCHEME_ADDITIVE = 0, BBX_SCHEME_SPLIT = 1 };

/* Cell models ("Cell models").  nvar and parameters:
 *  NONE    (1 var: V)             pure diffusion, no parameters;
 *  BARKLEY (2 vars: u, v)         params {a, b, eps}:  u' = u(1-u)(u-(v+b)/a)/eps,  v' = u - v;
 *  ZFK     (1 var: V)             params {alpha}:       V' = V(V-alpha)(1-V)  (eq (ZFKbidomV));
 *  FHN     (2 vars: u, v)         params {eps, beta, gamma}: u' = (u - u^3/3 - v)/eps,
 *                                  v' = eps(u + beta - gamma v)  (eq (FHN));
 *  CRN     (21 vars)              Courtemanche-Ramirez-Nattel 1998 atrial model, no
 *                                  parameters; state order V, Na_i, K_i, Ca_i, Ca_up, Ca_rel,
 *                                  m, h, j, oa, oi, ua, ui, xr, xs, d, f, fCa, u, v, w;
 *                                  the 15 gates use Rush-Larsen, the rest forward Euler;
 *  FK4     (4 vars: u, v, w, s)   params {tau_fi, tau_so1, tau_si, tau_w+} (epicardial
 *                                  0.11, 30.0181, 1.8875, 200 ms): the four-variable
 *                                  minimal model of the Fenton-Karma family (Bueno-Orovio,
 *                                  Cherry & Fenton 2008, epicardial set), u dimensionless;
 *                                  v, w, s use Rush-Larsen, u forward Euler;
 *  TP06    (19 vars)              ten Tusscher-Panfilov 2006 ventricular model, epicardial
 *                                  cell, no parameters; state order V, K_i, Na_i, Ca_i,
 *                                  Ca_ss, Ca_SR, Rbar, Xr1, Xr2, Xs, m, h, j, d, f, f2, fCass,
 *                                  s, r; the 12 gates use Rush-Larsen, the rest forward Euler. */
enum {
    BBX_MODEL_NONE = 0,
    BBX_MODEL_BARKLEY = 1,
    BBX_MODEL_ZFK = 2,
    BBX_MODEL_FHN = 3,
    BBX_MODEL_CRN = 4,
    BBX_MODEL_FK4 = 5,
    BBX_MODEL_TP06 = 6
};

/* What bbx_readout returns. */
enum {
    BBX_READ_VAR = 0,         /* double[nbox]: state variable `var`; void voxels NaN */
    BBX_READ_ACT_TIME = 1,    /* double[nbox]: activation time (ms); NaN if none / void */
    BBX_READ_APD90 = 2,       /* double[nbox]: APD90 (ms); NaN if not reached / void */
    BBX_READ_VMAX = 3,        /* double[nbox]: action-potential peak; NaN if not reached */
    BBX_READ_STATUS = 4,      /* uint8[nbox]: 0 resting, 1 rising, 2 repolarising,
                                 3 done; 255 void */
    BBX_READ_REDUCE_MAX = 5,  /* double[1]: max of `var` over tissue in `region` (FP64) */
    BBX_READ_REDUCE_SUM = 6,  /* double[1]: sum of `var` over tissue in `region` (FP64,
                                 fixed summation order: deterministic) */
    BBX_READ_NAN_FLAG = 7,    /* int32[1]: 1 if any state value is not finite */
    BBX_READ_STEP = 8,        /* int64[1]: number of steps taken (t = step * dt) */
    BBX_READ_WEIGHTS = 9,     /* double[nact*27]: the effective stencil weights W^p_q of
                                 every tissue voxel p (increasing box order), q = (dx,dy,dz)
                                 at (dz+1)*9 + (dy+1)*3 + (dx+1), centre = -sum of others */
    BBX_READ_FALLBACK_COUNT = 10, /* int64[1]: voxel updates that fell back from the
                                     surrogate to the plain kinetics since it was attached */
    BBX_READ_ECG = 11,            /* double[nelec]: pseudo-ECG of the current V at each
                                     electrode (bbx_ecg_set), computed now */
    BBX_READ_ECG_SERIES = 12,     /* double[count*nelec]: the sampled pseudo-ECG, sample-major */
    BBX_READ_ECG_COUNT = 13,      /* int64[1]: samples stored so far */
    BBX_READ_ALL_STATE = 14       /* double[nvar*nbox]: every state variable in box layout,
                                     variable after variable (void NaN): with BBX_READ_STEP a
                                     checkpoint, restored by bbx_state_set per variable and
                                     bbx_clock_set (the paper's `dump` / `load` of the state) */
};

/* Info queries for bbx_info.  SEND_* / RECV_*: values a slab grid (bbx_slab_create)
 * packs from its first / last own plane and unpacks into its lower / upper halo plane. */
enum { BBX_INFO_NACTIVE = 0, BBX_INFO_NVAR = 1, BBX_INFO_NBOX = 2, BBX_INFO_DEVICE_BYTES = 3,
       BBX_INFO_SEND_LO = 4, BBX_INFO_SEND_HI = 5, BBX_INFO_RECV_LO = 6, BBX_INFO_RECV_HI = 7 };

/*
 * Create a grid (the paper's `state` sentence with a geometry; "Format of
 * geometry files"): nx*ny*nz box (nz = 1 for 2D), spacing h > 0.
 *   mask   uint8[nbox], nonzero = tissue (grid indicator chi_p = 1); required.
 *   fibre  double[nbox*3] fibre direction per voxel (normalised here; void
 *          voxels ignored) or NULL for isotropic tissue with coefficient D_perp.
 *   D_par, D_perp  eigenvalues of D along / across the fibres (eq (sigma)), > 0.
 *   precision      BBX_FP32 or BBX_FP64.
 *   hip_stream     hipStream_t to enqueue on, or NULL.
 * Voxels outside the box count as void, which gives the no-flux condition at
 * the box faces too.  A tissue voxel whose fibre has length < 1e-12 gives
 * BBX_EINVAL, and so does a box of more than 2^31 - 1 voxels (box indices are
 * 32-bit).  Allocates device memory (two box-sized V arrays plus the per-tissue
 * state); *out receives the grid.
 */
int bbx_grid_create(int nx, int ny, int nz, double h, const uint8_t *mask, const double *fibre,
                    double D_par, double D_perp, int precision, void *hip_stream,
                    bbx_grid **out);

/* ------------------------------------------------------------------------
 * z-slab sub-domains ("Complex geometries and domain partitioning": the paper
 * splits the box into subdomains, one per process, that exchange boundary
 * layers of the diffusing variable every step).  Here a box is split along z
 * only: the only state a step reads from a neighbouring slab is V of the
 * adjacent plane (the 19-point stencil reaches one plane up and down, faces and
 * edges; every other variable is point-local), so one plane per side and step
 * is the whole exchange, and the paper's corner ordering for multi-axis splits
 * is not needed.  A slab grid is an ordinary grid (every other call works on
 * it) whose box is the slab's own planes plus one halo plane on each side.
 * ---------------------------------------------------------------------- */

/* Tissue-balanced split of the nz planes of a box into nslab (1..nz) slabs of
 * consecutive planes: z_bounds[nslab + 1] receives 0 = z_0 < z_1 < ... < z_nslab
 * = nz, each boundary the plane boundary nearest to where the tissue below it
 * reaches k/nslab of the total (every slab keeps at least one plane).  Host only;
 * mask as in bbx_grid_create.  Errors: BBX_EINVAL. */
int bbx_slab_bounds(int nx, int ny, int nz, const uint8_t *mask, int nslab, int *z_bounds);

/* Create the grid of the slab of global planes [z0, z1) of an nx*ny*nz box
 * (0 <= z0 < z1 <= nz): mask and fibre are the whole box's arrays (read, not
 * kept).  The slab grid's box has nz_s = z1 - z0 + 2 planes: plane 0 is global
 * plane z0 - 1, plane nz_s - 1 is global plane z1 (void where they lie outside
 * the global box); its own, stepped, voxels are the tissue of planes 1..nz_s-2,
 * and tissue in the two halo planes takes part in the stencil (geometry
 * included) exactly as in the whole box, so a step of every slab, with halo
 * planes holding the neighbours' V_n, gives bit for bit the whole box's step.
 * Every other entry point then works on the slab's box (host arrays have
 * nx*ny*nz_s entries; halo entries are never read as state, and read back as
 * NaN); pseudo-ECG electrode positions stay global (the slab's plane 0 lies at
 * z = (z0 - 1) h), so the slabs' ECGs sum to the whole box's.  Errors as
 * bbx_grid_create, plus BBX_EINVAL for a bad plane range. */
int bbx_slab_create(int nx, int ny, int nz, int z0, int z1, double h, const uint8_t *mask,
                    const double *fibre, double D_par, double D_perp, int precision,
                    void *hip_stream, bbx_grid **out);

/* Halo exchange of a slab grid, on its stream.  Pack copies the current V of the
 * tissue voxels of the first (side 0) or last (side 1) own plane, in increasing x
 * (fastest) and y order, into buf_dev (device, count values of the grid's
 * precision, count = bbx_info SEND_LO / SEND_HI).  Unpack writes count = RECV_LO
 * / RECV_HI values from buf_dev into the tissue voxels of the lower (side 0) or
 * upper (side 1) halo plane, same order.  Slab k's side-1 pack is slab k+1's
 * side-0 unpack and vice versa (the counts agree: both are the tissue of one
 * global plane).  Between two steps, every slab unpacks what its neighbours
 * packed after the previous step; a readout that applies the stencil (the
 * pseudo-ECG) needs the same exchange after the last step.  Errors: BBX_EINVAL
 * (side, count, NULL buffer), BBX_ESTATE (not a slab grid). */
int bbx_halo_pack(bbx_grid *g, int side, void *buf_dev, int64_t count);
int bbx_halo_unpack(bbx_grid *g, int side, const void *buf_dev, int64_t count);

/* Choose the cell model, its parameters (nparams must equal the model's count,
 * params may be NULL when it is 0), the time step dt > 0 and the scheme.
 * Allocates the model's state (initialised to 0 for every variable except V,
 * which keeps its values) and resets the step counter to 0.  Returns
 * BBX_EUNSTABLE if dt exceeds 2 / max_p sum_q |W^p_q| (Gershgorin bound of
 * the explicit diffusion step). */
int bbx_model_set(bbx_grid *g, int model, const double *params, int nparams, double dt,
                  int scheme);

/* Set state variable var (0 = V) from a host double[nbox] array; only tissue
 * entries are read.  Stream-ordered, the host array is copied before return. */
int bbx_state_set(bbx_grid *g, int var, const double *box_values);

/* Set state variable `var` to `value` on every tissue voxel (void entries of V
 * stay 0): the uniform initial condition of a large grid without a host array.
 * Errors as bbx_state_set, plus BBX_EINVAL for a non-finite value. */
int bbx_state_fill(bbx_grid *g, int var, double value);

/* Add a stimulus current (the external current term of eq (monodomain)):
 * amplitude (pA/pF; positive depolarises) applied to tissue voxels where
 * region[idx] != 0, during steps n with round(t_start/dt) + c*round(period/dt)
 * <= n < that + round(duration/dt), for c = 0 .. count-1 (period <= 0: once;
 * count <= 0 with period > 0: forever).  At most 32 stimuli; requires a model. */
int bbx_stimulus_add(bbx_grid *g, const uint8_t *region, double amplitude, double t_start,
                     double duration, double period, int count);

/* Remove all stimuli. */
int bbx_stimulus_clear(bbx_grid *g);

/* (Re)start activation-time / APD90 detection with threshold theta (the
 * paper's threshold-crossing recorder `k_poincare`, applied per voxel): the
 * current V becomes each voxel's rest level.  Per voxel, from each step's pair
 * (V_n, V_{n+1}): the first upward crossing of theta gives the activation time
 * (linear interpolation); the first decrease after it records the peak V_n;
 * the first downward crossing of rest + 0.1(peak - rest) after that gives
 * APD90 = crossing time - activation time.  theta NaN switches detection off. */
int bbx_recording_set(bbx_grid *g, double theta);

/* Check the state for non-finite values every `every` steps and at the end of
 * each bbx_step (every = 0 disables the check; the default is 1000).  With the
 * check on, bbx_step synchronises the stream at its end and returns
 * BBX_ENUMERIC if a value was not finite. */
int bbx_nan_check_set(bbx_grid *g, int64_t every);

/* Pseudo-ECG electrodes.  The library's pseudo-ECG of a field V at electrode
 * position x_e (mm) is
 *     phi(x_e) = h^3 sum_{p in tissue} (L V)_p / |x_p - x_e|,   x_p = h (x, y, z),
 * with L the step's own discrete diffusion operator (the weights of "Monodomain
 * diffusion and boundary conditions"): with no-flux boundaries, summation by
 * parts makes this the volume integral of -D grad V . grad(1/r) of the
 * classical pseudo-ECG (its constant factor left to the caller).  (L V)_p is
 * evaluated in the grid's precision; distances and all sums are FP64, reduced
 * in a fixed order (deterministic).  nelec (0..16) electrodes at xyz_mm[3*nelec]
 * (copied); no electrode may sit exactly on a tissue voxel centre (EINVAL).
 * every > 0: after each step that brings the step counter to a multiple of
 * `every`, the ECG of the new V is stored, up to max_samples samples (read with
 * BBX_READ_ECG_SERIES / _COUNT); every = 0: on demand only (BBX_READ_ECG).
 * Calling it again replaces the electrodes and clears stored samples; nelec = 0
 * turns the ECG off. */
int bbx_ecg_set(bbx_grid *g, int nelec, const double *xyz_mm, int64_t every, int64_t max_samples);

/* Rush-Larsen tabulation ("Exponential solvers": the rate coefficients of
 * gates that depend on V alone are precomputed on a grid of V at start time):
 * dv > 0 makes an FP32 CRN grid read every voltage-only kinetic term (for the
 * twelve voltage-gated gates y_inf and e^{-dt/tau}; six voltage factors of
 * currents) from a table over [-120, 80] mV with spacing dv, evaluated in FP64
 * and interpolated linearly (V outside the range is clamped).  The table is
 * rebuilt by bbx_model_set.  dv = 0 returns to direct evaluation.  Other
 * models or FP64 grids: BBX_ENOTSUP. */
int bbx_tabulation_set(bbx_grid *g, double dv);

/* Integrator of the kinetics ("Kinetics solvers"): EULER_RL (the default) advances
 * concentrations and recovery variables by forward Euler (eq (Euler)) and gates by
 * Rush-Larsen (eqs (RL), (RLcoeff)); RK4 is the classical fourth-order Runge-Kutta
 * scheme (the paper's `rk4` solver for cases where accuracy matters) applied to every
 * state variable of a voxel, gates included (dg/dt = (g_inf - g)/tau), with the
 * stimulus current -- and in the additive scheme the diffusion term L V -- held at its
 * step-n value through the four stages; in the split scheme it starts from V* = V +
 * dt L V.  RK4 costs four evaluations of the kinetics per step and uses the tissue-list
 * kernel with cached accesses on every grid; tabulated CRN terms are ignored under RK4.
 * Like every explicit scheme it is only conditionally stable: a gate with time constant
 * tau needs dt below about 2.8 tau (TP06's sodium activation, tau ~1e-3 ms near rest,
 * diverges at dt = 0.005 ms), where Rush-Larsen is stable at any dt.  Kept until changed.  Errors: BBX_EINVAL (unknown integrator), BBX_ENOTSUP (RK4 with
 * a surrogate attached). */
enum { BBX_INTEGRATOR_EULER_RL = 0, BBX_INTEGRATOR_RK4 = 1 };
int bbx_integrator_set(bbx_grid *g, int integrator);

/* Set the step counter (t = step * dt), e.g. when resuming from a checkpoint
 * read with BBX_READ_VAR / BBX_READ_STEP; step >= 0. */
int bbx_clock_set(bbx_grid *g, int64_t step);

/* Launch mode of bbx_step: chunk = 0 launches every step directly (the default);
 * chunk = K > 0 (even, <= 4096) replays a HIP graph of K step launches whenever at least K
 * steps are left, the rest launched directly.  The graph's kernels read the step number
 * from a device counter (set from the host clock at each bbx_step call, advanced by the
 * graph's last node) and evaluate their stimulus windows and t_n from it with the host's
 * arithmetic, so results are bitwise those of direct launches.  Graphs are captured on
 * first use and dropped by any call that changes what a step does (model, stimuli,
 * recording, tabulation, integrator, surrogate attach or detach, this call).  With a
 * surrogate attached the graph holds both of its launches per step.  Steps stay direct
 * while pseudo-ECG samples are being taken; with the finite check on, it runs after
 * each chunk that crosses a multiple of its interval.  Errors: BBX_EINVAL (chunk),
 * BBX_ENOTSUP (a grid created on the null stream: capture needs a stream of its own). */
int bbx_graph_set(bbx_grid *g, int chunk);

/* Advance nsteps >= 0 time steps (one fused kernel launch per step). */
int bbx_step(bbx_grid *g, int64_t nsteps);

/* Read results.  `var` selects the state variable for VAR and REDUCE_*;
 * `region` (uint8[nbox] or NULL = all tissue) restricts REDUCE_*.  out must
 * hold out_bytes >= the size listed for `what`.  out_on_device = 1: out is a
 * device pointer and the copy is stream-ordered (asynchronous);
 * out_on_device = 0: host pointer, the call synchronises the stream. */
int bbx_readout(bbx_grid *g, int what, int var, const uint8_t *region, void *out,
                size_t out_bytes, int out_on_device);

/* ------------------------------------------------------------------------
 * Surrogate ionic map.  A network nin -> 128 -> 128 -> nout with SiLU
 * activations stands in for the kinetic one-step map of the explicit scheme,
 * (V, g) -> (V + dt(-I_ion(V, g)), g+) (eq (Euler) with Rush-Larsen gates,
 * eqs (RL), (RLcoeff)), on normalised inputs x = (s - mu_in) * in_scale and
 * normalised increments d = ((s+ - s) - mu_out) / sigma_out.  Weights are
 * kept in FP32 (master) and BF16 (the copies the MFMA kernels read);
 * activations are BF16, accumulation FP32.  Parameters use the flat layout
 * W1[128][nin], b1[128], W2[128][128], b2[128], W3[nout][128], b3[nout].
 * ---------------------------------------------------------------------- */
typedef struct bbx_mlp bbx_mlp;

/* Create a network (1 <= nin, nout <= 32) with weights drawn from a seeded
 * counter-based generator (uniform, scaled by 1/sqrt(fan_in)), biases 0,
 * identity normalisation and zero Adam moments.  Work is enqueued on
 * hip_stream (NULL = null stream). */
int bbx_mlp_create(int nin, int nout, uint64_t seed, void *hip_stream, bbx_mlp **out);

/* Copy the FP32 master parameters (count = number of parameters) to the host
 * (set = 0) or from the host (set = 1; refreshes the BF16 copies). */
int bbx_mlp_params(bbx_mlp *m, int set, float *host, size_t count);

/* Copy the normalisation [4][32] = in_mean, in_scale, out_mean, out_sigma to
 * (set = 0) or from (set = 1) the host; out_sigma must be >= 0. */
int bbx_mlp_norm(bbx_mlp *m, int set, float *host);

/* Fit the normalisation to training pairs on the device: S [n][nin] states
 * and S1 [n][nout] the states one step later (row-major per sample; nin must
 * equal nout).  Sets in_mean/in_scale from the states (in_scale 1 for a
 * constant state) and out_mean/out_sigma from the increments S1 - S
 * (out_sigma 0 for a constant increment, which is then predicted exactly as
 * out_mean; e.g. K_i in FP32, whose change per step is below its rounding).  If stats
 * is not NULL it receives double[7][32]: mean, std, min, max of the states,
 * then mean, std, max |.| of the increments. */
int bbx_mlp_fit_norm(bbx_mlp *m, const float *S_dev, const float *S1_dev, int64_t n,
                     double *stats);

/* Network outputs for n normalised inputs X [n][nin] (device) into Y [n][nout]
 * (device): the raw network, no normalisation applied. */
int bbx_mlp_forward(bbx_mlp *m, const float *X_dev, int64_t n, float *Y_dev);

/* Mean-squared-error loss over the n samples and nout outputs of
 * (network(X) - T), X [n][nin], T [n][nout] on the device, and its gradient
 * with respect to the parameters, left in the network for bbx_mlp_adam and
 * copied to grad_host (nparams floats) if not NULL.  n <= 65536. */
int bbx_mlp_grad(bbx_mlp *m, const float *X_dev, const float *T_dev, int64_t n, float *grad_host,
                 double *loss);

/* The gradient of bbx_mlp_grad without any device allocation, for callers that
 * cannot allocate: code under HIP graph capture, tight training loops, harnesses
 * that forbid hipMalloc.  Same loss and gradient (same kernels, same summation
 * order) for 1 <= n <= 4096 samples; larger n gives BBX_EINVAL.  X_dev [n][nin] and
 * T_dev [n][nout] are device inputs; the gradient stays in the network for
 * bbx_mlp_adam and is also copied to grad_dev (nparams floats, device) and the
 * loss to loss_dev (one double, device) when those are not NULL.  Stream-ordered on
 * the network's stream, no synchronisation.  The training scratch is one static
 * device array of 5.6 MiB per GPU (kept until the process ends) shared by every
 * call on that GPU: calls that overlap on one GPU (other streams or threads) race.
 * The network's device must be the current device. */
int bbx_mlp_grad_static(bbx_mlp *m, const float *X_dev, const float *T_dev, int64_t n,
                        float *grad_dev, double *loss_dev);

/* One Adam step (bias-corrected) with the last gradient. */
int bbx_mlp_adam(bbx_mlp *m, float lr, float beta1, float beta2, float eps);

/* Train on raw pairs (S, S1 as in bbx_mlp_fit_norm, normalised with the
 * network's current normalisation): iters minibatch Adam steps of `batch`
 * samples (<= 65536) drawn with replacement by a counter-based generator.
 * loss_hist (iters floats, may be NULL) receives each step's batch loss. */
int bbx_mlp_train(bbx_mlp *m, const float *S_dev, const float *S1_dev, int64_t n, int64_t batch,
                  int64_t iters, float lr, uint64_t seed, float *loss_hist);

/* Shift the output biases so that the network maps the state s0 (nin floats,
 * device) exactly to the increment s1 - s0 (s1 on the device): e.g. s0 = a
 * resting state and s1 = its plain one-step image, which makes the resting
 * state an exact fixed point of the surrogate map as it is of the plain one.
 * Requires nin == nout. */
int bbx_mlp_anchor(bbx_mlp *m, const float *s0_dev, const float *s1_dev);

/* Free the network. */
void bbx_mlp_destroy(bbx_mlp *m);

/* Write the state of n tissue voxels drawn uniformly with replacement (seeded
 * counter-based generator) to out [n][nvar] (device, FP32). */
int bbx_sample_states(bbx_grid *g, int64_t n, uint64_t seed, float *out_dev);

/* Apply the grid's plain kinetic one-step map (model, parameters and dt; no
 * diffusion, no stimulus) to n states in [n][nvar] (device, FP32) -> out. */
int bbx_ionic_map(bbx_grid *g, const float *in_dev, int64_t n, float *out_dev);

/* Attach a trained network as the kinetics of an FP32 grid (NULL detaches).
 * nin = nout = the model's nvar.  Each step then gives the plain kinetic
 * update to every tissue voxel whose kinetic input leaves [lo, hi] (nvar
 * floats each), evaluates the network for the others, and falls back to the
 * plain update for a voxel whose predicted gates leave [-1e-3, 1 + 1e-3]
 * (accepted gates are clamped to [0, 1]), whose predicted |dV| exceeds dv_max,
 * or whose prediction is not finite.  A fallback voxel gets exactly the plain
 * step's arithmetic.  Supported models: Barkley, FHN, CRN, TP06.  The
 * network's weights are copied; it may be destroyed after. */
int bbx_surrogate_set(bbx_grid *g, const bbx_mlp *m, const float *lo, const float *hi,
                      float dv_max);

/* Phase singularities in z cross-sections (the `singz` device of "Input/output and
 * visualization": intersections of isolines of two fields, the isolines' pieces in
 * each grid cell from linear interpolation).  Fields: state variables var_u and var_v
 * of the grid (0 = V), levels u_level and v_level.  A cell is the square of four
 * tissue voxels (x..x+1, y..y+1) of one z plane; a corner is above a level when its
 * value is >= the level; an isoline crosses a cell edge whose corners differ, at the
 * linearly interpolated point; two crossed edges give one piece, four (a saddle) give
 * two, which separate the corner pair whose class differs from that of the four
 * corners' mean; each crossing of a u piece with a v piece is a point.
 *   stats [7] (host): count, mean x, y, z, standard deviation (population) of x, y,
 *         z, coordinates in mm (x_p = h (x, y, z)), from FP64 sums in a fixed order
 *         (deterministic);  a slab grid searches its own planes only and reports global
 *         coordinates (z of the whole box), so the slabs' points together are the box's;
 *   points (host, may be NULL): the first min(count, max_points) points, [k][3] mm,
 *         in an order that varies from run to run (sort to compare);
 *   npoints (may be NULL): the number of points found.
 * Synchronises the stream; allocates temporaries (and, on a sparse grid's first
 * call, a 4-byte-per-voxel box-to-tissue map kept with the grid).  Errors:
 * BBX_EINVAL (variables, levels, max_points), BBX_ESTATE (no model). */
int bbx_tips(bbx_grid *g, int var_u, double u_level, int var_v, double v_level, double *stats,
             double *points, int64_t max_points, int64_t *npoints);

/* Attach a surrogate from host arrays (a network trained elsewhere) instead of a
 * bbx_mlp: nin = nout = the model's nvar; weights_bf16 holds W1[128][nin], W2[128][128],
 * W3[nout][128] one after the other as BF16 bit patterns (the precision the MFMA kernels
 * read), biases b1[128], b2[128], b3[nout] (FP32), norm[4][32] = in_mean, in_scale,
 * out_mean, out_sigma (as bbx_mlp_norm); lo, hi, dv_max as bbx_surrogate_set, whose
 * semantics the attached network then has.  Arrays are copied.  Errors as
 * bbx_surrogate_set, plus BBX_EINVAL for non-finite parameters or a negative
 * out_sigma. */
int bbx_surrogate_import(bbx_grid *g, int nin, int nout, const uint16_t *weights_bf16,
                         const float *biases, const float *norm, const float *lo, const float *hi,
                         float dv_max);

/* Integer facts about a grid (BBX_INFO_*). */
int bbx_info(const bbx_grid *g, int what, int64_t *out);

/* Free the grid and all its device memory (synchronises its stream). */
void bbx_grid_destroy(bbx_grid *g);

/* Message of the calling thread's last error ("" if none). */
const char *bbx_last_error(void);

/* ------------------------------------------------------------------------
 * Batched ensemble: many independent 2D rectangular tissues advanced together
 * by one launch per step (the same explicit scheme as a grid: the anisotropic
 * no-flux 9-point stencil of "Monodomain diffusion and boundary conditions"
 * with a tissue-uniform tensor, fused with the kinetics of "Kinetics solvers",
 * additive coupling, rectangular stimuli, activation/APD90 recording).  Each
 * tissue has its own size, diffusion coefficients, fibre angle and model
 * parameters; the model and dt are common.  All tissues live in one set of
 * device arrays, tissue after tissue, each x-fastest; a step launches one
 * workgroup per (tissue, tile) of a tile shape chosen by bbx_ensemble_tune.
 * Steps are launched either directly or by replaying a captured HIP graph of
 * a fixed number of steps (bbx_ensemble_graph_set).  Conventions as above;
 * an ensemble is not thread-safe.
 * ------------------------------------------------------------------------ */
typedef struct bbx_ensemble bbx_ensemble;

/* Tile variants of the ensemble step (bbx_ensemble_variant_set / _tune):
 * LDS-staged tiles of 64x4, 32x8 or 16x16 voxels; 64x4 tiles that read
 * neighbours straight from memory; or 64-column strips of 32 or 128 rows that
 * each wave marches row by row (x neighbours from adjacent lanes, the next row
 * loaded while the current one is computed). */
enum { BBX_ENS_TILE_64x4 = 0, BBX_ENS_TILE_32x8 = 1, BBX_ENS_TILE_16x16 = 2,
       BBX_ENS_DIRECT_64x4 = 3, BBX_ENS_MARCH_64x32 = 4, BBX_ENS_MARCH_64x128 = 5,
       BBX_ENS_NVARIANT = 6 };

/* Info queries for bbx_ensemble_info. */
enum { BBX_ENS_INFO_VOXELS = 0, BBX_ENS_INFO_TILES = 1, BBX_ENS_INFO_VARIANT = 2,
       BBX_ENS_INFO_DEVICE_BYTES = 3, BBX_ENS_INFO_GRAPH_CHUNK = 4, BBX_ENS_INFO_NVAR = 5 };

/*
 * Create an ensemble of ntissue >= 1 tissues.  Tissue i is an nx[i] x ny[i]
 * rectangle of tissue (every voxel active; no-flux at its edges) with grid
 * step h (mm), tensor D = Dperp[i] I + (Dpar[i] - Dperp[i]) f f^T (eq (sigma))
 * for the in-plane unit fibre f = (cos angle[i], sin angle[i]) (radians),
 * kinetics `model` (BBX_MODEL_NONE, _BARKLEY, _ZFK, _FHN or _FK4) with
 * parameters params[i*nparams .. i*nparams + nparams-1] (nparams = the model's
 * count), time step dt (ms) and precision BBX_FP32/BBX_FP64.  Every state
 * variable starts at 0.  hip_stream: the stream all work is enqueued on; NULL
 * makes the ensemble create (and own) a stream of its own, since graph capture
 * needs a non-null stream.  Errors: BBX_EINVAL (sizes < 1, more than 2^31
 * voxels in total, non-finite or negative coefficients, wrong nparams),
 * BBX_ENOTSUP (model CRN), BBX_EUNSTABLE (dt above the Gershgorin bound of
 * some tissue), BBX_ENOMEM / BBX_EDEVICE. */
int bbx_ensemble_create(int ntissue, const int *nx, const int *ny, double h,
                        const double *Dpar, const double *Dperp, const double *angle,
                        int model, const double *params, int nparams, double dt,
                        int precision, void *hip_stream, bbx_ensemble **out);

/* Set state variable `var` of tissue `tissue` from values[nx*ny] (x fastest).
 * Errors: BBX_EINVAL (index out of range, NULL values). */
int bbx_ensemble_state_set(bbx_ensemble *e, int tissue, int var, const double *values);

/* Add a stimulus to tissue `tissue` over the voxel rectangle x0 <= x < x1,
 * y0 <= y < y1: amplitude added to du/dt while on, windows as in
 * bbx_stimulus_add (whole steps, round half away from zero; period 0 = once;
 * count 0 = unlimited).  At most 8 stimuli per tissue.  Errors: BBX_EINVAL. */
int bbx_ensemble_stimulus_add(bbx_ensemble *e, int tissue, int x0, int x1, int y0, int y1,
                              double amplitude, double t_start, double duration,
                              double period, int count);

/* Start activation / APD90 recording at threshold theta on every tissue (as
 * bbx_recording_set; V_rest = each voxel's value now). */
int bbx_ensemble_recording_set(bbx_ensemble *e, double theta);

/* Launch mode of bbx_ensemble_step: chunk = 0 launches every step directly;
 * chunk = K > 0 (even, <= 4096) captures K steps into a HIP graph on first use
 * and replays it, launching any remainder directly.  Results are bitwise the
 * same either way.  The graph is recaptured after any change to the ensemble.
 * Errors: BBX_EINVAL. */
int bbx_ensemble_graph_set(bbx_ensemble *e, int chunk);

/* Select a tile variant (BBX_ENS_TILE_* / BBX_ENS_DIRECT_*).  All variants
 * compute bitwise-identical results. */
int bbx_ensemble_variant_set(bbx_ensemble *e, int variant);

/* Autotune: time `steps` steps of every variant on a scratch copy of the
 * current state (the ensemble's own state and clock are untouched), select
 * the fastest and return it in *variant (may be NULL); times_ms[BBX_ENS_NVARIANT] (may be
 * NULL) receives each variant's time.  Synchronises the stream. */
int bbx_ensemble_tune(bbx_ensemble *e, int steps, int *variant, double *times_ms);

/* Advance every tissue by nsteps >= 0 steps (asynchronous). */
int bbx_ensemble_step(bbx_ensemble *e, int64_t nsteps);

/* Copy a result of tissue `tissue` to host memory out[count]: BBX_READ_VAR
 * (var; nx*ny doubles), BBX_READ_ACT_TIME, BBX_READ_APD90, BBX_READ_VMAX (nx*ny
 * doubles, NaN where not reached), BBX_READ_STATUS (nx*ny bytes),
 * BBX_READ_NAN_FLAG (int32[1], over the whole ensemble), BBX_READ_STEP
 * (int64[1]).  count is the number of elements of out; it must be at least
 * what the request returns.  Synchronises the stream.  Errors: BBX_EINVAL,
 * BBX_ESTATE (recording results before bbx_ensemble_recording_set). */
int bbx_ensemble_readout(bbx_ensemble *e, int what, int tissue, int var, void *out, size_t count);

/* Integer facts about an ensemble (BBX_ENS_INFO_*). */
int bbx_ensemble_info(const bbx_ensemble *e, int what, int64_t *out);

/* Free the ensemble, its graph, its device memory and any stream it created
 * (synchronises its stream). */
void bbx_ensemble_destroy(bbx_ensemble *e);

#ifdef __cplusplus
}
#endif

#endif /* BBX_H */
