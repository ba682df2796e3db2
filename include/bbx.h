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
 *                                  the 15 gates use Rush-Larsen, the rest forward Euler. */
enum {
    BBX_MODEL_NONE = 0,
    BBX_MODEL_BARKLEY = 1,
    BBX_MODEL_ZFK = 2,
    BBX_MODEL_FHN = 3,
    BBX_MODEL_CRN = 4
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
    BBX_READ_WEIGHTS = 9      /* double[nact*27]: the effective stencil weights W^p_q of
                                 every tissue voxel p (increasing box order), q = (dx,dy,dz)
                                 at (dz+1)*9 + (dy+1)*3 + (dx+1), centre = -sum of others */
};

/* Info queries for bbx_info. */
enum { BBX_INFO_NACTIVE = 0, BBX_INFO_NVAR = 1, BBX_INFO_NBOX = 2, BBX_INFO_DEVICE_BYTES = 3 };

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
 * BBX_EINVAL.  Allocates device memory; *out receives the grid.
 */
int bbx_grid_create(int nx, int ny, int nz, double h, const uint8_t *mask, const double *fibre,
                    double D_par, double D_perp, int precision, void *hip_stream,
                    bbx_grid **out);

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

/* Set the step counter (t = step * dt), e.g. when resuming from a checkpoint
 * read with BBX_READ_VAR / BBX_READ_STEP; step >= 0. */
int bbx_clock_set(bbx_grid *g, int64_t step);

/* Advance nsteps >= 0 time steps (one fused kernel launch per step). */
int bbx_step(bbx_grid *g, int64_t nsteps);

/* Read results.  `var` selects the state variable for VAR and REDUCE_*;
 * `region` (uint8[nbox] or NULL = all tissue) restricts REDUCE_*.  out must
 * hold out_bytes >= the size listed for `what`.  out_on_device = 1: out is a
 * device pointer and the copy is stream-ordered (asynchronous);
 * out_on_device = 0: host pointer, the call synchronises the stream. */
int bbx_readout(bbx_grid *g, int what, int var, const uint8_t *region, void *out,
                size_t out_bytes, int out_on_device);

/* Integer facts about a grid (BBX_INFO_*). */
int bbx_info(const bbx_grid *g, int what, int64_t *out);

/* Free the grid and all its device memory (synchronises its stream). */
void bbx_grid_destroy(bbx_grid *g);

/* Message of the calling thread's last error ("" if none). */
const char *bbx_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* BBX_H */
