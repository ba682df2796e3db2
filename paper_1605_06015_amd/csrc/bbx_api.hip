// Host side of libbbx: argument validation, one-off geometry preprocessing in
// FP64, device allocation, per-step launch sequencing and readout.  Every
// entry point catches everything: no C++ exception crosses the C ABI.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/bbx.h"
#include "bbx_internal.h"
#include "mlp_internal.h"

using namespace bbx;

namespace {

thread_local std::string g_err;

// Host-side log on stderr, on when the environment variable BBX_LOG is set to a
// non-zero value when the library first logs: set-up calls and every failed call.
bool log_on()
{
    static const bool on = [] {
        const char *v = getenv("BBX_LOG");
        return v && *v && strcmp(v, "0") != 0;
    }();
    return on;
}

void log_line(const char *fmt, ...)
{
    if (!log_on()) return;
    char buf[640];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    fprintf(stderr, "bbx: %s\n", buf);
}

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    log_line("error %d: %s", code, buf);
    return code;
}

int hip_fail(hipError_t e, const char *what)
{
    return fail(e == hipErrorOutOfMemory ? BBX_ENOMEM : BBX_EDEVICE, "%s: %s", what,
                hipGetErrorString(e));
}

#define HIP_TRY(expr, what)                      \
    do {                                         \
        hipError_t e_ = (expr);                  \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

int model_nvar(int m)
{
    switch (m) {
    case BBX_MODEL_NONE: return 1;
    case BBX_MODEL_BARKLEY: return 2;
    case BBX_MODEL_ZFK: return 1;
    case BBX_MODEL_FHN: return 2;
    case BBX_MODEL_CRN: return 21;
    case BBX_MODEL_FK4: return 4;
    case BBX_MODEL_TP06: return 19;
    default: return -1;
    }
}

int model_nparams(int m)
{
    switch (m) {
    case BBX_MODEL_NONE: return 0;
    case BBX_MODEL_BARKLEY: return 3;
    case BBX_MODEL_ZFK: return 1;
    case BBX_MODEL_FHN: return 3;
    case BBX_MODEL_CRN: return 0;
    case BBX_MODEL_FK4: return 4;
    case BBX_MODEL_TP06: return 0;
    default: return -1;
    }
}

// Nearest integer, halves away from zero (the rounding of stimulus windows).
int64_t steps_of(double t, double dt) { return (int64_t)llround(t / dt); }

struct DevBuf {
    void *p = nullptr;
    ~DevBuf() { if (p) (void)hipFree(p); }
};

}  // namespace

struct StimDef {
    double amp, t0, dur, period;
    int count;
};

struct bbx_grid {
    int nx = 0, ny = 0, nz = 0;
    int64_t nbox = 0, nact = 0, pitch = 0;
    double h = 0, Dpar = 0, Dperp = 0;
    int prec = 0, es = 4;
    int aniso = 0, dense = 0;
    hipStream_t stream = nullptr;
    double wsum_max = 0;  // max_p sum_q |W^p_q| including the centre

    int32_t *d_idx = nullptr;
    uint32_t *d_nbr = nullptr;
    void *d_geo = nullptr;
    void *d_V[2] = {nullptr, nullptr};
    int cur = 0;
    void *d_st = nullptr;
    int st_alloc = 0;  // variables allocated in d_st

    int model = -1, nvar = 1, scheme = 0;
    int integrator = 0;                // BBX_INTEGRATOR_*
    double dt = 0, prm[kMaxParams] = {};

    std::vector<StimDef> stims;
    std::vector<uint32_t> h_stimbits;
    uint32_t *d_stimbits = nullptr;
    void *d_stimamp = nullptr;

    int rec = 0;
    double theta = NAN;
    uint8_t *d_status = nullptr;
    void *d_at = nullptr, *d_vmax = nullptr, *d_apd = nullptr, *d_vrep = nullptr;

    int64_t n = 0, nan_every = 1000;
    double tab_dv = 0;                 // > 0: CRN voltage-only terms from a table
    float *d_tab = nullptr;
    int tab_n = 0;
    // attached surrogate (FP32 grids): network copy, accepted box, network list
    int sur = 0;
    MlpDev snet = {};
    float *d_slo = nullptr, *d_shi = nullptr;
    float dv_max = 0;
    int32_t *d_acc_list = nullptr, *d_acc_cnt = nullptr;   // network list segments, lengths
    unsigned long long *d_fb = nullptr;                      // fallback counts per segment
    int sur_nblk = 0;                                        // list segments (classifier workgroups)
    double *d_parts = nullptr, *d_red = nullptr;
    int *d_flag = nullptr;
    // pseudo-ECG sampling
    EcgElectrodes ecg = {};
    int64_t ecg_every = 0, ecg_max = 0, ecg_count = 0;
    double *d_ecg_series = nullptr, *d_ecg_parts = nullptr, *d_ecg_now = nullptr;
    int nparts = 1024;
    size_t bytes = 0;
    // z-slab sub-domain (bbx_slab_create): box planes 0 and nz-1 are halo planes of the
    // neighbouring slabs; zoff = global z of plane 0.  side 0 = lower, 1 = upper.
    int slab = 0, zoff = 0;
    int64_t send_n[2] = {0, 0}, recv_n[2] = {0, 0};
    int32_t *d_send[2] = {nullptr, nullptr}, *d_recv[2] = {nullptr, nullptr};
    int32_t *d_map = nullptr;          // box -> tissue index (-1 void), built on first use
    // graph replay of bbx_step (bbx_graph_set): chunk steps per graph, one graph per
    // starting V buffer; device step counter and stimulus windows
    int chunk = 0;
    hipGraph_t graph[2] = {nullptr, nullptr};
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    int64_t *d_nbase = nullptr;
    StimWin *d_win = nullptr;
    bool win_dirty = true;
};

namespace {

template <typename P>
hipError_t dalloc(bbx_grid *g, P **p, size_t bytes)
{
    void *q = nullptr;
    hipError_t e = hipMalloc(&q, bytes ? bytes : 1);
    if (e == hipSuccess) {
        *p = (P *)q;
        g->bytes += bytes;
    }
    return e;
}

void dfree(void *p)
{
    if (p) (void)hipFree(p);
}

void graph_drop(bbx_grid *g)
{
    for (int c = 0; c < 2; c++) {
        if (g->gexec[c]) (void)hipGraphExecDestroy(g->gexec[c]);
        if (g->graph[c]) (void)hipGraphDestroy(g->graph[c]);
        g->gexec[c] = nullptr;
        g->graph[c] = nullptr;
    }
    g->win_dirty = true;
}

void free_all(bbx_grid *g)
{
    graph_drop(g);
    void *ps[] = {g->d_idx, g->d_nbr, g->d_geo, g->d_V[0], g->d_V[1], g->d_st,
                  g->d_stimbits, g->d_stimamp, g->d_status, g->d_at, g->d_vmax, g->d_apd,
                  g->d_vrep, g->d_parts, g->d_red, g->d_flag, g->d_slo, g->d_shi,
                  g->d_acc_list, g->d_acc_cnt, g->d_fb, g->d_tab, g->d_ecg_series, g->d_ecg_parts, g->d_ecg_now, g->snet.w1, g->snet.w2, g->snet.w3,
                  g->snet.bias, g->snet.norm, g->d_send[0], g->d_send[1], g->d_recv[0],
                  g->d_recv[1], g->d_map, g->d_nbase, g->d_win};
    for (void *p : ps) dfree(p);
}

// Unit fibre at a box voxel (caller checked it is tissue and normalisable).
inline void unit_fibre(const double *fib, int64_t idx, double f[3])
{
    const double *v = fib + 3 * idx;
    const double n = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    f[0] = v[0] / n;
    f[1] = v[1] / n;
    f[2] = v[2] / n;
}

inline void tensor(const double f[3], double Dpar, double Dperp, double D[3][3])
{
    for (int j = 0; j < 3; j++)
        for (int k = 0; k < 3; k++) D[j][k] = (j == k ? Dperp : 0.0) + (Dpar - Dperp) * f[j] * f[k];
}

template <typename T>
StepArgs<T> make_args(const bbx_grid *g)
{
    StepArgs<T> a;
    memset(&a, 0, sizeof a);
    a.nx = g->nx;
    a.ny = g->ny;
    a.nz = g->nz;
    a.dense = g->dense;
    a.nact = g->nact;
    a.pitch = g->pitch;
    a.idx = g->d_idx;
    a.nbr = g->d_nbr;
    a.geo = (const T *)g->d_geo;
    a.Dpar = (T)g->Dpar;
    a.Dperp = (T)g->Dperp;
    a.ih2 = (T)(1.0 / (g->h * g->h));
    a.st = (T *)g->d_st;
    for (int i = 0; i < kMaxParams; i++) a.prm[i] = (T)g->prm[i];
    a.dt = (T)g->dt;
    a.split = g->scheme == BBX_SCHEME_SPLIT;
    a.rk4 = g->integrator == BBX_INTEGRATOR_RK4;
    a.tab = (g->tab_dv > 0 && g->model == BBX_MODEL_CRN && g->prec == BBX_FP32) ? g->d_tab : nullptr;
    a.nstim = (int)g->stims.size();
    a.stimbits = g->d_stimbits;
    a.stim_amp = (const T *)g->d_stimamp;
    a.rec = g->rec;
    a.theta = (T)g->theta;
    a.status = g->d_status;
    a.at = (T *)g->d_at;
    a.vmax = (T *)g->d_vmax;
    a.apd = (T *)g->d_apd;
    a.vrep = (T *)g->d_vrep;
    // Measured: streaming accesses take 13% off the TP06 step on the 512x512x384 double
    // shell (403 MB box, 1.9 GB state), 3% off the dense 512x512x384 stencil and 1.4% off
    // a 300^3 CRN box (108 MB box, 2.3 GB state), and slow the cases that fit the cache
    // (CRN cup: 4 MB box, 31 MB state; thin shell: 77 MB box, 128 MB state).
    a.nt = (double)g->nbox * sizeof(T) > kInfinityCacheBytes ||
           (double)g->nact * (g->nvar - 1) * sizeof(T) > kInfinityCacheBytes;
    if (a.rk4) a.nt = 0;               // the RK4 kernels use cached accesses only
    // Dense boxes with light kinetics (<= 4 variables) use the z-marching LDS kernel;
    // with the 19/21-variable models the one-voxel-per-thread kernel is faster
    // (measured on a 300^3 CRN box: 1.02 vs 1.12 ms per step), and a.zc = 0 selects it.
    if (g->dense && g->nvar <= 4 && !a.rk4) {
        a.gx = (g->nx + kTileX - 1) / kTileX;
        a.gy = (g->ny + kTileY - 1) / kTileY;
        // z-chunk: long enough to amortise the two extra halo planes, short enough
        // to give every SIMD several workgroups
        int zc = 16;   // measured best on the 512x512x384 box (8, 32, 64+ are slower)
        while (zc > 4 && (int64_t)a.gx * a.gy * ((g->nz + zc - 1) / zc) < 8192) zc /= 2;
        a.zc = zc;
        a.nblk = a.gx * a.gy * ((g->nz + zc - 1) / zc);
    } else {
        a.zc = 0;
        const int wg = a.nt ? kStreamBlock : kBlock;   // the tissue-list kernel's workgroup
        a.nblk = (int)((g->nact + wg - 1) / wg);
    }
    a.per_xcd = (a.nblk + kXcd - 1) / kXcd;
    return a;
}

uint32_t stim_mask(const bbx_grid *g, int64_t n)
{
    uint32_t m = 0;
    for (size_t k = 0; k < g->stims.size(); k++) {
        const StimDef &s = g->stims[k];
        const int64_t n0 = steps_of(s.t0, g->dt), len = steps_of(s.dur, g->dt);
        const int64_t per = s.period > 0 ? steps_of(s.period, g->dt) : 0;
        if (n < n0 || len <= 0) continue;
        const int64_t r = n - n0;
        bool on;
        if (per <= 0) {
            on = r < len;
        } else {
            const int64_t c = r / per;
            on = !(s.count > 0 && c >= s.count) && (r - c * per) < len;
        }
        if (on) m |= 1u << k;
    }
    return m;
}

// (Re)build the CRN voltage table for the current dt (FP32 CRN grids with tabulation on).
int build_table(bbx_grid *g)
{
    if (!(g->tab_dv > 0) || g->model != BBX_MODEL_CRN || g->prec != BBX_FP32) return BBX_OK;
    const int n = (int)ceil((kTabVmax - kTabVmin) / g->tab_dv) + 1;
    if (n != g->tab_n) {
        dfree(g->d_tab);
        g->d_tab = nullptr;
        g->tab_n = 0;
        hipError_t e = dalloc(g, &g->d_tab, (size_t)(n + 1) * kTabWidth * sizeof(float));
        if (e != hipSuccess) return hip_fail(e, "hipMalloc");
        g->tab_n = n;
    }
    HIP_TRY(launch_crn_table(kTabVmin, g->tab_dv, n, g->dt, g->d_tab, g->stream), "table");
    return BBX_OK;
}

SurArgs sur_args(const bbx_grid *g)
{
    SurArgs su;
    su.net = g->snet;
    su.lo = g->d_slo;
    su.hi = g->d_shi;
    su.dv_max = g->dv_max;
    su.acc_list = g->d_acc_list;
    su.acc_cnt = g->d_acc_cnt;
    su.fb = g->d_fb;
    su.nblk = g->sur_nblk;
    return su;
}

// Capture one chunk of steps starting from V buffer c: each step reads its number from the
// device counter (base + position) and evaluates its stimuli and t_n there; the last node
// advances the counter by the chunk.
template <typename T>
int graph_capture(bbx_grid *g, int c)
{
    StepArgs<T> a = make_args<T>(g);
    a.nbase = g->d_nbase;
    a.win = g->d_win;
    a.dt64 = g->dt;
    HIP_TRY(hipStreamBeginCapture(g->stream, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
    hipError_t e = hipSuccess;
    for (int j = 0; j < g->chunk && e == hipSuccess; j++) {
        a.Vin = (const T *)g->d_V[c ^ (j & 1)];
        a.Vout = (T *)g->d_V[c ^ (j & 1) ^ 1];
        a.jstep = j;
        bool done = false;
        if constexpr (std::is_same<T, float>::value) {
            if (g->sur) {
                StepArgs<float> b = a;
                b.nblk = (int)((g->nact + kBlock - 1) / kBlock);
                b.per_xcd = (b.nblk + kXcd - 1) / kXcd;
                e = launch_surrogate_step(g->model, g->aniso, b, sur_args(g), g->stream);
                done = true;
            }
        }
        if (!done) e = launch_step<T>(g->model, g->aniso, a, g->stream);
    }
    if (e == hipSuccess) e = launch_counter(g->d_nbase, g->chunk, 1, g->stream);
    hipGraph_t gr = nullptr;
    const hipError_t e2 = hipStreamEndCapture(g->stream, &gr);
    if (e != hipSuccess || e2 != hipSuccess) {
        if (gr) (void)hipGraphDestroy(gr);
        return hip_fail(e != hipSuccess ? e : e2, "graph capture");
    }
    g->graph[c] = gr;
    e = hipGraphInstantiate(&g->gexec[c], gr, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(gr);
        g->graph[c] = nullptr;
        g->gexec[c] = nullptr;
        return hip_fail(e, "hipGraphInstantiate");
    }
    return BBX_OK;
}

// Replay whole chunks while at least one is left; returns the steps done.  Not used while
// pseudo-ECG samples are being taken (those steps stay direct).
template <typename T>
int graph_steps(bbx_grid *g, int64_t nsteps, int64_t *done)
{
    *done = 0;
    if (g->chunk <= 0 || nsteps < g->chunk || g->nact == 0) return BBX_OK;
    if (g->ecg_every > 0 && g->ecg_count < g->ecg_max) return BBX_OK;
    hipError_t e = hipSuccess;
    if (!g->d_nbase && (e = dalloc(g, &g->d_nbase, sizeof(int64_t))) != hipSuccess) return hip_fail(e, "hipMalloc");
    if (!g->d_win && (e = dalloc(g, &g->d_win, kMaxStim * sizeof(StimWin))) != hipSuccess) return hip_fail(e, "hipMalloc");
    if (g->win_dirty) {
        StimWin w[kMaxStim] = {};
        for (size_t k = 0; k < g->stims.size(); k++) {
            const StimDef &sd = g->stims[k];
            w[k] = {steps_of(sd.t0, g->dt), steps_of(sd.dur, g->dt),
                    sd.period > 0 ? steps_of(sd.period, g->dt) : 0, (int64_t)sd.count};
        }
        // ordered after the replays still in flight on the grid's stream (which read the
        // old table), and finished before w goes out of scope
        HIP_TRY(hipMemcpyAsync(g->d_win, w, sizeof w, hipMemcpyHostToDevice, g->stream), "hipMemcpyAsync");
        HIP_TRY(hipStreamSynchronize(g->stream), "hipStreamSynchronize");
        g->win_dirty = false;
    }
    HIP_TRY(launch_counter(g->d_nbase, g->n, 0, g->stream), "counter");
    const int nst = g->nvar - 1;
    while (nsteps - *done >= g->chunk) {
        const int c = g->cur;
        if (!g->gexec[c]) {
            int rc = graph_capture<T>(g, c);
            if (rc) return rc;
        }
        HIP_TRY(hipGraphLaunch(g->gexec[c], g->stream), "hipGraphLaunch");
        const int64_t n0 = g->n;
        g->n += g->chunk;                  // chunk even: the V buffer parity is unchanged
        *done += g->chunk;
        if (g->nan_every > 0 && n0 / g->nan_every != g->n / g->nan_every)
            HIP_TRY(launch_nonfinite<T>((const T *)g->d_V[g->cur], g->d_idx, g->dense, (const T *)g->d_st,
                                        nst, g->nact, g->pitch, g->d_flag, g->stream), "finite check");
    }
    return BBX_OK;
}

template <typename T>
int step_impl(bbx_grid *g, int64_t nsteps)
{
    StepArgs<T> a = make_args<T>(g);
    const int nst = g->nvar - 1;
    // a fill kernel, not a memset: a caller may capture bbx_step into a graph
    if (g->nan_every > 0) HIP_TRY(launch_fill<int>(g->d_flag, 0, 1, g->stream), "flag clear");
    int64_t done = 0;
    int rc = graph_steps<T>(g, nsteps, &done);
    if (rc) return rc;
    nsteps -= done;
    for (int64_t s = 0; s < nsteps; s++) {
        const int64_t n = g->n;
        a.Vin = (const T *)g->d_V[g->cur];
        a.Vout = (T *)g->d_V[g->cur ^ 1];
        a.stim_on = g->stims.empty() ? 0u : stim_mask(g, n);
        a.tn = (T)((double)n * g->dt);
        if (g->nact > 0) {
            bool done = false;
            if constexpr (std::is_same<T, float>::value) {
                if (g->sur) {
                    StepArgs<float> b = a;
                    b.nblk = (int)((g->nact + kBlock - 1) / kBlock);   // classifier: one thread per voxel
                    b.per_xcd = (b.nblk + kXcd - 1) / kXcd;
                    const SurArgs su = sur_args(g);
                    HIP_TRY(launch_surrogate_step(g->model, g->aniso, b, su, g->stream), "surrogate step");
                    done = true;
                }
            }
            if (!done) HIP_TRY(launch_step<T>(g->model, g->aniso, a, g->stream), "step launch");
        }
        g->cur ^= 1;
        g->n = n + 1;                  // clock and buffer parity stay consistent on errors
        if (g->ecg_every > 0 && (n + 1) % g->ecg_every == 0 && g->ecg_count < g->ecg_max && g->nact > 0) {
            StepArgs<T> b = a;
            b.Vin = (const T *)g->d_V[g->cur];
            HIP_TRY(launch_ecg<T>(b, g->aniso, g->ecg, g->d_ecg_parts,
                                  g->d_ecg_series + g->ecg_count * g->ecg.n, g->stream), "pseudo-ECG");
            g->ecg_count++;
        }
        if (g->nan_every > 0 && (n + 1) % g->nan_every == 0)
            HIP_TRY(launch_nonfinite<T>((const T *)g->d_V[g->cur], g->d_idx, g->dense,
                                        (const T *)g->d_st, nst, g->nact, g->pitch, g->d_flag,
                                        g->stream),
                    "finite check");
    }
    if (g->nan_every > 0) {
        HIP_TRY(launch_nonfinite<T>((const T *)g->d_V[g->cur], g->d_idx, g->dense,
                                    (const T *)g->d_st, nst, g->nact, g->pitch, g->d_flag,
                                    g->stream),
                "finite check");
        int flag = 0;
        HIP_TRY(hipMemcpyAsync(&flag, g->d_flag, sizeof(int), hipMemcpyDeviceToHost, g->stream),
                "hipMemcpyAsync");
        HIP_TRY(hipStreamSynchronize(g->stream), "hipStreamSynchronize");
        if (flag) return fail(BBX_ENUMERIC, "non-finite state value after step %lld",
                              (long long)g->n);
    }
    return BBX_OK;
}

// Host array of T from doubles, in tissue order or box order (void = 0).
template <typename T>
std::vector<T> convert(const bbx_grid *g, const std::vector<int64_t> *act, const double *src,
                       int box_order)
{
    std::vector<T> out(box_order ? (size_t)g->nbox : (size_t)g->nact, T(0));
    for (int64_t t = 0; t < g->nact; t++) {
        const int64_t b = act ? (*act)[t] : t;
        out[box_order ? b : t] = (T)src[b];
    }
    return out;
}

std::vector<int64_t> tissue_list(const bbx_grid *g, const int32_t *h_idx)
{
    std::vector<int64_t> act((size_t)g->nact);
    for (int64_t t = 0; t < g->nact; t++) act[t] = g->dense ? t : h_idx[t];
    return act;
}

int download_idx(const bbx_grid *g, std::vector<int32_t> &h_idx)
{
    h_idx.clear();
    if (g->dense) return BBX_OK;
    h_idx.resize((size_t)g->nact);
    HIP_TRY(hipMemcpyAsync(h_idx.data(), g->d_idx, g->nact * sizeof(int32_t),
                           hipMemcpyDeviceToHost, g->stream), "hipMemcpyAsync");
    HIP_TRY(hipStreamSynchronize(g->stream), "hipStreamSynchronize");
    return BBX_OK;
}

// Tissue mask (box order) rebuilt from the tissue list.
int download_mask(const bbx_grid *g, std::vector<uint8_t> &mask)
{
    mask.assign((size_t)g->nbox, g->dense ? 1 : 0);
    if (g->dense) return BBX_OK;
    std::vector<int32_t> h_idx;
    int rc = download_idx(g, h_idx);
    if (rc) return rc;
    for (int32_t b : h_idx) mask[(size_t)b] = 1;
    return BBX_OK;
}

// Geometry preprocessing.  Tissue voxels of the box planes [own0, own1) are the grid's
// own (stepped) voxels; tissue in other planes (a slab's halo planes) only takes part as
// neighbours.
template <typename T>
int create_impl(bbx_grid *g, const uint8_t *mask, const double *fibre, int own0, int own1)
{
    // tissue list (increasing box order)
    const int64_t nxy = (int64_t)g->nx * g->ny;
    const int64_t b0 = own0 * nxy, b1 = own1 * nxy;
    int64_t count = 0;
    for (int64_t b = b0; b < b1; b++) count += mask[b] != 0;
    std::vector<int32_t> idx;
    idx.reserve((size_t)count);
    for (int64_t b = b0; b < b1; b++)
        if (mask[b]) idx.push_back((int32_t)b);
    g->nact = (int64_t)idx.size();
    g->dense = g->nact == g->nbox;
    g->pitch = (g->nact + 63) / 64 * 64;

    auto tissue = [&](int x, int y, int z) -> bool {
        if (x < 0 || y < 0 || z < 0 || x >= g->nx || y >= g->ny || z >= g->nz) return false;
        return mask[(int64_t)x + (int64_t)g->nx * ((int64_t)y + (int64_t)g->ny * z)] != 0;
    };

    std::vector<uint32_t> nbr((size_t)g->nact);
    std::vector<T> geo;
    if (g->aniso) geo.assign((size_t)(6 * g->nact), T(0));
    const double ih2 = 1.0 / (g->h * g->h);
    double wmax = 0;
    for (int64_t t = 0; t < g->nact; t++) {
        const int64_t b = idx[t];
        const int x = (int)(b % g->nx), y = (int)((b / g->nx) % g->ny);
        const int z = (int)(b / ((int64_t)g->nx * g->ny));
        uint32_t bits = 0;
        for (int k = 0; k < 18; k++) {
            const NbOff o = nb_off(k);
            if (tissue(x + o.dx, y + o.dy, z + o.dz)) bits |= 1u << k;
        }
        nbr[t] = bits;
        double D[3][3] = {{g->Dperp, 0, 0}, {0, g->Dperp, 0}, {0, 0, g->Dperp}};
        double c[3] = {0, 0, 0};
        if (g->aniso) {
            double f[3];
            unit_fibre(fibre, b, f);
            tensor(f, g->Dpar, g->Dperp, D);
            // Tensor-gradient face coefficient: both face neighbours along k must be
            // tissue; D at a void neighbour p +- q_j is replaced by D^p.
            double Dn[3][2][3][3];
            for (int j = 0; j < 3; j++)
                for (int sgn = 0; sgn < 2; sgn++) {
                    const NbOff o = nb_off(2 * j + sgn);
                    if ((bits >> (2 * j + sgn)) & 1u) {
                        double fn[3];
                        unit_fibre(fibre, b + o.dx + (int64_t)g->nx * (o.dy + (int64_t)g->ny * o.dz), fn);
                        tensor(fn, g->Dpar, g->Dperp, Dn[j][sgn]);
                    } else {
                        memcpy(Dn[j][sgn], D, sizeof D);
                    }
                }
            for (int k = 0; k < 3; k++) {
                if (((bits >> (2 * k)) & 3u) != 3u) continue;
                double sdiv = 0;
                for (int j = 0; j < 3; j++) sdiv += Dn[j][0][j][k] - Dn[j][1][j][k];
                c[k] = 0.25 * ih2 * sdiv;
            }
            for (int k = 0; k < 3; k++) {
                geo[6 * t + k] = (T)f[k];
                geo[6 * t + 3 + k] = (T)c[k];
            }
        }
        // Gershgorin radius of row p: |W_0| + sum |W_q| <= 2 sum |W_q|
        double s = 0;
        for (int k = 0; k < 18; k++) {
            if (!((bits >> k) & 1u)) continue;
            if (k < 6) {
                const int ax = k / 2;
                s += fabs(D[ax][ax] * ih2 + ((k & 1) ? -c[ax] : c[ax]));
            } else if (g->aniso) {
                const int plane = (k - 6) / 4;
                const int j = plane == 2 ? 1 : 0, kk = plane == 0 ? 1 : 2;
                s += fabs(0.5 * D[j][kk] * ih2);
            }
        }
        wmax = fmax(wmax, 2.0 * s);
    }
    g->wsum_max = wmax;

    const size_t es = sizeof(T);
    hipError_t e = hipSuccess;
    if (!g->dense) {
        if ((e = dalloc(g, &g->d_idx, g->nact * sizeof(int32_t))) != hipSuccess) return hip_fail(e, "hipMalloc");
        if ((e = dalloc(g, &g->d_nbr, g->nact * sizeof(uint32_t))) != hipSuccess) return hip_fail(e, "hipMalloc");
        HIP_TRY(hipMemcpy(g->d_idx, idx.data(), g->nact * sizeof(int32_t), hipMemcpyHostToDevice), "hipMemcpy");
        HIP_TRY(hipMemcpy(g->d_nbr, nbr.data(), g->nact * sizeof(uint32_t), hipMemcpyHostToDevice), "hipMemcpy");
    }
    if (g->aniso) {
        if ((e = dalloc(g, &g->d_geo, 6 * g->nact * es)) != hipSuccess) return hip_fail(e, "hipMalloc");
        if (g->nact)
            HIP_TRY(hipMemcpy(g->d_geo, geo.data(), 6 * g->nact * es, hipMemcpyHostToDevice), "hipMemcpy");
    }
    for (int k = 0; k < 2; k++) {
        if ((e = dalloc(g, &g->d_V[k], g->nbox * es)) != hipSuccess) return hip_fail(e, "hipMalloc");
        HIP_TRY(hipMemset(g->d_V[k], 0, g->nbox * es), "hipMemset");
    }
    if ((e = dalloc(g, &g->d_parts, g->nparts * sizeof(double))) != hipSuccess) return hip_fail(e, "hipMalloc");
    if ((e = dalloc(g, &g->d_red, 8 * sizeof(double))) != hipSuccess) return hip_fail(e, "hipMalloc");
    if ((e = dalloc(g, &g->d_flag, sizeof(int))) != hipSuccess) return hip_fail(e, "hipMalloc");
    if ((e = dalloc(g, &g->d_stimamp, kMaxStim * es)) != hipSuccess) return hip_fail(e, "hipMalloc");
    HIP_TRY(hipMemset(g->d_stimamp, 0, kMaxStim * es), "hipMemset");
    return BBX_OK;
}

template <typename T>
int alloc_state(bbx_grid *g, int nvar)
{
    const int need = nvar - 1;
    if (need != g->st_alloc) {
        dfree(g->d_st);
        g->d_st = nullptr;
        g->st_alloc = 0;
        if (need > 0) {
            hipError_t e = dalloc(g, &g->d_st, (size_t)need * g->pitch * sizeof(T));
            if (e != hipSuccess) return hip_fail(e, "hipMalloc");
            g->st_alloc = need;
        }
    }
    if (need > 0)
        HIP_TRY(launch_fill<T>((T *)g->d_st, T(0), (int64_t)need * g->pitch, g->stream), "fill");
    return BBX_OK;
}

template <typename T>
int state_set_impl(bbx_grid *g, int var, const double *vals)
{
    std::vector<int32_t> h_idx;
    int rc = download_idx(g, h_idx);
    if (rc) return rc;
    std::vector<int64_t> act = tissue_list(g, h_idx.data());
    if (var == 0) {
        std::vector<T> box = convert<T>(g, &act, vals, 1);
        HIP_TRY(hipMemcpyAsync(g->d_V[g->cur], box.data(), g->nbox * sizeof(T),
                               hipMemcpyHostToDevice, g->stream), "hipMemcpyAsync");
        HIP_TRY(hipStreamSynchronize(g->stream), "hipStreamSynchronize");
    } else {
        std::vector<T> lst = convert<T>(g, &act, vals, 0);
        T *dst = (T *)g->d_st + (int64_t)(var - 1) * g->pitch;
        HIP_TRY(hipMemcpyAsync(dst, lst.data(), g->nact * sizeof(T), hipMemcpyHostToDevice,
                               g->stream), "hipMemcpyAsync");
        HIP_TRY(hipStreamSynchronize(g->stream), "hipStreamSynchronize");
    }
    return BBX_OK;
}

template <typename T>
int state_fill_impl(bbx_grid *g, int var, double value)
{
    if (var == 0) {
        if (g->dense) HIP_TRY(launch_fill<T>((T *)g->d_V[g->cur], (T)value, g->nbox, g->stream), "fill");
        else HIP_TRY(launch_fill_tissue<T>((T *)g->d_V[g->cur], g->d_idx, g->nact, (T)value, g->stream), "fill");
    } else {
        HIP_TRY(launch_fill<T>((T *)g->d_st + (int64_t)(var - 1) * g->pitch, (T)value, g->nact, g->stream), "fill");
    }
    HIP_TRY(hipStreamSynchronize(g->stream), "hipStreamSynchronize");
    return BBX_OK;
}

template <typename T>
int recording_impl(bbx_grid *g, double theta)
{
    const size_t es = sizeof(T);
    if (!g->d_status) {
        hipError_t e;
        if ((e = dalloc(g, &g->d_status, g->nact ? g->nact : 1)) != hipSuccess) return hip_fail(e, "hipMalloc");
        void **ps[] = {&g->d_at, &g->d_vmax, &g->d_apd, &g->d_vrep};
        for (void **p : ps)
            if ((e = dalloc(g, p, g->pitch * es)) != hipSuccess) return hip_fail(e, "hipMalloc");
    }
    const T nan = (T)NAN;
    HIP_TRY(launch_fill<uint8_t>(g->d_status, 0, g->nact, g->stream), "fill");
    HIP_TRY(launch_fill<T>((T *)g->d_at, nan, g->nact, g->stream), "fill");
    HIP_TRY(launch_fill<T>((T *)g->d_vmax, nan, g->nact, g->stream), "fill");
    HIP_TRY(launch_fill<T>((T *)g->d_apd, nan, g->nact, g->stream), "fill");
    HIP_TRY(launch_gather<T>((const T *)g->d_V[g->cur], g->d_idx, g->dense, g->nact,
                             (T *)g->d_vrep, g->stream), "gather");
    g->theta = theta;
    g->rec = 1;
    return BBX_OK;
}

template <typename T>
int readout_impl(bbx_grid *g, int what, int var, const uint8_t *region, void *out,
                 size_t out_bytes, int on_dev)
{
    const int64_t nbox = g->nbox;
    switch (what) {
    case BBX_READ_VAR:
    case BBX_READ_ACT_TIME:
    case BBX_READ_APD90:
    case BBX_READ_VMAX: {
        if (out_bytes < (size_t)nbox * sizeof(double)) return fail(BBX_EINVAL, "out_bytes too small");
        const T *src;
        int is_box = 0;
        if (what == BBX_READ_VAR) {
            if (var < 0 || var >= g->nvar) return fail(BBX_EINVAL, "var %d out of range", var);
            if (var == 0) { src = (const T *)g->d_V[g->cur]; is_box = 1; }
            else src = (const T *)g->d_st + (int64_t)(var - 1) * g->pitch;
        } else {
            if (!g->d_status) return fail(BBX_ESTATE, "recording was never started");
            src = (const T *)(what == BBX_READ_ACT_TIME ? g->d_at : what == BBX_READ_APD90 ? g->d_apd : g->d_vmax);
        }
        if (on_dev) {
            HIP_TRY(launch_to_box<T>(src, is_box, g->d_idx, g->dense, g->nact, nbox, (double *)out, g->stream), "to_box");
            return BBX_OK;
        }
        DevBuf tmp;
        HIP_TRY(hipMalloc(&tmp.p, nbox * sizeof(double)), "hipMalloc");
        HIP_TRY(launch_to_box<T>(src, is_box, g->d_idx, g->dense, g->nact, nbox, (double *)tmp.p, g->stream), "to_box");
        HIP_TRY(hipMemcpyAsync(out, tmp.p, nbox * sizeof(double), hipMemcpyDeviceToHost, g->stream), "hipMemcpyAsync");
        HIP_TRY(hipStreamSynchronize(g->stream), "hipStreamSynchronize");
        return BBX_OK;
    }
    case BBX_READ_STATUS: {
        if (on_dev) return fail(BBX_ENOTSUP, "STATUS is read to host memory only");
        if (!g->d_status) return fail(BBX_ESTATE, "recording was never started");
        if (out_bytes < (size_t)nbox) return fail(BBX_EINVAL, "out_bytes too small");
        std::vector<uint8_t> st((size_t)g->nact);
        std::vector<int32_t> h_idx;
        int rc = download_idx(g, h_idx);
        if (rc) return rc;
        if (g->nact) {
            HIP_TRY(hipMemcpyAsync(st.data(), g->d_status, g->nact, hipMemcpyDeviceToHost, g->stream), "hipMemcpyAsync");
            HIP_TRY(hipStreamSynchronize(g->stream), "hipStreamSynchronize");
        }
        uint8_t *o = (uint8_t *)out;
        memset(o, 255, (size_t)nbox);
        for (int64_t t = 0; t < g->nact; t++) o[g->dense ? t : h_idx[t]] = st[t];
        return BBX_OK;
    }
    case BBX_READ_REDUCE_MAX:
    case BBX_READ_REDUCE_SUM: {
        if (out_bytes < sizeof(double)) return fail(BBX_EINVAL, "out_bytes too small");
        if (var < 0 || var >= g->nvar) return fail(BBX_EINVAL, "var %d out of range", var);
        const T *src = var == 0 ? (const T *)g->d_V[g->cur] : (const T *)g->d_st + (int64_t)(var - 1) * g->pitch;
        DevBuf reg;
        if (region) {
            HIP_TRY(hipMalloc(&reg.p, nbox), "hipMalloc");
            HIP_TRY(hipMemcpyAsync(reg.p, region, nbox, hipMemcpyHostToDevice, g->stream), "hipMemcpyAsync");
        }
        HIP_TRY(launch_reduce<T>(src, var == 0, g->d_idx, g->dense, g->nact, (const uint8_t *)reg.p,
                                 what == BBX_READ_REDUCE_SUM, g->d_parts, g->nparts, g->d_red, g->stream),
                "reduce");
        HIP_TRY(hipMemcpyAsync(out, g->d_red, sizeof(double),
                               on_dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, g->stream),
                "hipMemcpyAsync");
        HIP_TRY(hipStreamSynchronize(g->stream), "hipStreamSynchronize");
        return BBX_OK;
    }
    case BBX_READ_NAN_FLAG: {
        if (on_dev) return fail(BBX_ENOTSUP, "NAN_FLAG is read to host memory only");
        if (out_bytes < sizeof(int32_t)) return fail(BBX_EINVAL, "out_bytes too small");
        HIP_TRY(hipMemsetAsync(g->d_flag, 0, sizeof(int), g->stream), "hipMemsetAsync");
        HIP_TRY(launch_nonfinite<T>((const T *)g->d_V[g->cur], g->d_idx, g->dense, (const T *)g->d_st,
                                    g->nvar - 1, g->nact, g->pitch, g->d_flag, g->stream), "finite check");
        HIP_TRY(hipMemcpyAsync(out, g->d_flag, sizeof(int32_t), hipMemcpyDeviceToHost, g->stream), "hipMemcpyAsync");
        HIP_TRY(hipStreamSynchronize(g->stream), "hipStreamSynchronize");
        return BBX_OK;
    }
    case BBX_READ_FALLBACK_COUNT: {
        if (on_dev) return fail(BBX_ENOTSUP, "FALLBACK_COUNT is read to host memory only");
        if (out_bytes < sizeof(int64_t)) return fail(BBX_EINVAL, "out_bytes too small");
        unsigned long long v = 0;
        if (g->d_fb && g->sur_nblk > 0) {
            std::vector<unsigned long long> fb((size_t)g->sur_nblk);
            HIP_TRY(hipMemcpyAsync(fb.data(), g->d_fb, fb.size() * sizeof(unsigned long long),
                                   hipMemcpyDeviceToHost, g->stream), "hipMemcpyAsync");
            HIP_TRY(hipStreamSynchronize(g->stream), "hipStreamSynchronize");
            for (unsigned long long x : fb) v += x;
        }
        int64_t o = (int64_t)v;
        memcpy(out, &o, sizeof o);
        return BBX_OK;
    }
    case BBX_READ_STEP: {
        if (on_dev) return fail(BBX_ENOTSUP, "STEP is read to host memory only");
        if (out_bytes < sizeof(int64_t)) return fail(BBX_EINVAL, "out_bytes too small");
        memcpy(out, &g->n, sizeof(int64_t));
        return BBX_OK;
    }
    case BBX_READ_WEIGHTS: {
        const size_t need = (size_t)g->nact * 27 * sizeof(double);
        if (out_bytes < need) return fail(BBX_EINVAL, "out_bytes too small");
        StepArgs<T> a = make_args<T>(g);
        if (on_dev) {
            HIP_TRY(launch_weights<T>(a, g->aniso, (double *)out, g->stream), "weights");
            return BBX_OK;
        }
        DevBuf tmp;
        HIP_TRY(hipMalloc(&tmp.p, need ? need : 1), "hipMalloc");
        HIP_TRY(launch_weights<T>(a, g->aniso, (double *)tmp.p, g->stream), "weights");
        if (need) HIP_TRY(hipMemcpyAsync(out, tmp.p, need, hipMemcpyDeviceToHost, g->stream), "hipMemcpyAsync");
        HIP_TRY(hipStreamSynchronize(g->stream), "hipStreamSynchronize");
        return BBX_OK;
    }
    case BBX_READ_ECG: {
        if (g->ecg.n <= 0) return fail(BBX_ESTATE, "no electrodes (bbx_ecg_set)");
        if (out_bytes < (size_t)g->ecg.n * sizeof(double)) return fail(BBX_EINVAL, "out_bytes too small");
        if (g->nact == 0) return fail(BBX_EINVAL, "the grid has no tissue");
        StepArgs<T> a = make_args<T>(g);
        a.Vin = (const T *)g->d_V[g->cur];
        HIP_TRY(launch_ecg<T>(a, g->aniso, g->ecg, g->d_ecg_parts, g->d_ecg_now, g->stream), "pseudo-ECG");
        HIP_TRY(hipMemcpyAsync(out, g->d_ecg_now, g->ecg.n * sizeof(double),
                               on_dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, g->stream),
                "hipMemcpyAsync");
        HIP_TRY(hipStreamSynchronize(g->stream), "hipStreamSynchronize");
        return BBX_OK;
    }
    case BBX_READ_ECG_SERIES: {
        if (g->ecg.n <= 0) return fail(BBX_ESTATE, "no electrodes (bbx_ecg_set)");
        const size_t need = (size_t)g->ecg_count * g->ecg.n * sizeof(double);
        if (out_bytes < need) return fail(BBX_EINVAL, "out_bytes too small");
        if (need)
            HIP_TRY(hipMemcpyAsync(out, g->d_ecg_series, need,
                                   on_dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, g->stream),
                    "hipMemcpyAsync");
        HIP_TRY(hipStreamSynchronize(g->stream), "hipStreamSynchronize");
        return BBX_OK;
    }
    case BBX_READ_ALL_STATE: {
        // every state variable in box layout, variable after variable (a checkpoint: with
        // BBX_READ_STEP it restores through bbx_state_set and bbx_clock_set)
        const size_t need = (size_t)g->nvar * nbox * sizeof(double);
        if (out_bytes < need) return fail(BBX_EINVAL, "out_bytes too small");
        DevBuf tmp;
        double *dst = (double *)out;
        if (!on_dev) {
            HIP_TRY(hipMalloc(&tmp.p, need), "hipMalloc");
            dst = (double *)tmp.p;
        }
        for (int v = 0; v < g->nvar; v++) {
            const T *src = v == 0 ? (const T *)g->d_V[g->cur] : (const T *)g->d_st + (int64_t)(v - 1) * g->pitch;
            HIP_TRY(launch_to_box<T>(src, v == 0, g->d_idx, g->dense, g->nact, nbox, dst + (int64_t)v * nbox,
                                     g->stream), "to_box");
        }
        if (!on_dev) {
            HIP_TRY(hipMemcpyAsync(out, tmp.p, need, hipMemcpyDeviceToHost, g->stream), "hipMemcpyAsync");
            HIP_TRY(hipStreamSynchronize(g->stream), "hipStreamSynchronize");
        }
        return BBX_OK;
    }
    case BBX_READ_ECG_COUNT: {
        if (on_dev) return fail(BBX_ENOTSUP, "ECG_COUNT is read to host memory only");
        if (out_bytes < sizeof(int64_t)) return fail(BBX_EINVAL, "out_bytes too small");
        memcpy(out, &g->ecg_count, sizeof(int64_t));
        return BBX_OK;
    }
    default:
        return fail(BBX_EINVAL, "unknown readout %d", what);
    }
}

}  // namespace

// ============================================================================ C ABI

// Error state shared with the other entry-point files of the library.
int bbx::api_error(int code, const char *msg)
{
    g_err = msg;
    log_line("error %d: %s", code, msg);
    return code;
}

void bbx::api_log(const char *msg) { log_line("%s", msg); }

void bbx::api_clear_error() { g_err.clear(); }

extern "C" {

const char *bbx_last_error(void) { return g_err.c_str(); }

}  // extern "C"

namespace {

// Shared by bbx_grid_create and bbx_slab_create: validate, build, and on success hand
// the grid to *out.  Box planes [own0, own1) hold the grid's own voxels.
int grid_create_common(int nx, int ny, int nz, double h, const uint8_t *mask, const double *fibre,
                       double D_par, double D_perp, int precision, void *hip_stream, int own0,
                       int own1, bbx_grid **out)
{
    if (!out) return fail(BBX_EINVAL, "out is NULL");
    *out = nullptr;
    if (nx < 1 || ny < 1 || nz < 1) return fail(BBX_EINVAL, "box sizes must be >= 1");
    const int64_t nbox = (int64_t)nx * ny * nz;
    if (nbox > 2147483647LL) return fail(BBX_EINVAL, "box has more than 2^31-1 voxels");
    if (!(h > 0) || !isfinite(h)) return fail(BBX_EINVAL, "h must be positive");
    if (!(D_par > 0) || !(D_perp > 0) || !isfinite(D_par) || !isfinite(D_perp))
        return fail(BBX_EINVAL, "D_par and D_perp must be positive");
    if (precision != BBX_FP32 && precision != BBX_FP64) return fail(BBX_EINVAL, "bad precision");
    if (!mask) return fail(BBX_EINVAL, "mask is NULL");
    if (fibre) {
        for (int64_t b = 0; b < nbox; b++) {
            if (!mask[b]) continue;
            const double *v = fibre + 3 * b;
            const double n = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
            if (!(n >= 1e-12) || !isfinite(n))
                return fail(BBX_EINVAL, "tissue voxel %lld has a non-normalisable fibre", (long long)b);
        }
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return fail(BBX_EDEVICE, "no HIP device");

    bbx_grid *g = new bbx_grid();
    g->nx = nx; g->ny = ny; g->nz = nz; g->nbox = nbox;
    g->h = h; g->Dpar = D_par; g->Dperp = D_perp;
    g->prec = precision; g->es = precision == BBX_FP64 ? 8 : 4;
    g->aniso = fibre != nullptr && D_par != D_perp;
    g->stream = (hipStream_t)hip_stream;
    int rc = precision == BBX_FP64 ? create_impl<double>(g, mask, fibre, own0, own1)
                                   : create_impl<float>(g, mask, fibre, own0, own1);
    if (rc != BBX_OK) {
        std::string keep = g_err;
        free_all(g);
        delete g;
        g_err = keep;
        return rc;
    }
    g->h_stimbits.assign((size_t)g->nact, 0u);
    log_line("grid %p: %dx%dx%d box, %lld tissue voxels (%s), %s, %s, planes [%d, %d) own, "
             "explicit diffusion dt bound %g ms", (void *)g, nx, ny, nz, (long long)g->nact,
             g->dense ? "dense" : "tissue list", g->aniso ? "anisotropic" : "isotropic",
             precision == BBX_FP64 ? "FP64" : "FP32", own0, own1,
             g->wsum_max > 0 ? 2.0 / g->wsum_max : 0.0);
    *out = g;
    return BBX_OK;
}

// Box indices of the tissue voxels of box plane z, x fastest.
std::vector<int32_t> plane_tissue(const bbx_grid *g, const uint8_t *mask, int z)
{
    std::vector<int32_t> v;
    const int64_t nxy = (int64_t)g->nx * g->ny;
    for (int64_t i = 0; i < nxy; i++)
        if (mask[z * nxy + i]) v.push_back((int32_t)(z * nxy + i));
    return v;
}

}  // namespace

extern "C" {

int bbx_grid_create(int nx, int ny, int nz, double h, const uint8_t *mask, const double *fibre,
                    double D_par, double D_perp, int precision, void *hip_stream, bbx_grid **out)
{
    try {
        g_err.clear();
        return grid_create_common(nx, ny, nz, h, mask, fibre, D_par, D_perp, precision, hip_stream,
                                  0, nz, out);
    } catch (...) {
        return fail(BBX_ENOMEM, "host allocation failed");
    }
}

int bbx_slab_bounds(int nx, int ny, int nz, const uint8_t *mask, int nslab, int *z_bounds)
{
    try {
        g_err.clear();
        if (nx < 1 || ny < 1 || nz < 1) return fail(BBX_EINVAL, "box sizes must be >= 1");
        if (!mask || !z_bounds) return fail(BBX_EINVAL, "NULL argument");
        if (nslab < 1 || nslab > nz) return fail(BBX_EINVAL, "nslab must be in [1, nz]");
        const int64_t nxy = (int64_t)nx * ny;
        std::vector<int64_t> cum((size_t)nz + 1, 0);      // tissue in planes [0, z)
        for (int z = 0; z < nz; z++) {
            int64_t c = 0;
            for (int64_t i = 0; i < nxy; i++) c += mask[z * nxy + i] != 0;
            cum[z + 1] = cum[z] + c;
        }
        const int64_t total = cum[nz];
        z_bounds[0] = 0;
        for (int k = 1; k < nslab; k++) {
            // the first plane boundary at which the tissue below reaches k/nslab of the
            // total, kept at least one plane above the previous boundary and leaving at
            // least one plane for each slab still to come
            const double target = (double)total * k / nslab;
            int z = z_bounds[k - 1] + 1;
            while (z < nz - (nslab - k) && (double)cum[z] < target) z++;
            // the nearer of z - 1 and z to the target
            if (z - 1 > z_bounds[k - 1] && target - (double)cum[z - 1] < (double)cum[z] - target) z--;
            z_bounds[k] = z;
        }
        z_bounds[nslab] = nz;
        return BBX_OK;
    } catch (...) {
        return fail(BBX_ENOMEM, "host allocation failed");
    }
}

int bbx_slab_create(int nx, int ny, int nz, int z0, int z1, double h, const uint8_t *mask,
                    const double *fibre, double D_par, double D_perp, int precision,
                    void *hip_stream, bbx_grid **out)
{
    try {
        g_err.clear();
        if (out) *out = nullptr;
        if (nx < 1 || ny < 1 || nz < 1) return fail(BBX_EINVAL, "box sizes must be >= 1");
        if (!mask) return fail(BBX_EINVAL, "mask is NULL");
        if (z0 < 0 || z1 > nz || z0 >= z1) return fail(BBX_EINVAL, "need 0 <= z0 < z1 <= nz");
        const int L = z1 - z0, ns = L + 2;
        const int64_t nxy = (int64_t)nx * ny;
        if (nxy * ns > 2147483647LL) return fail(BBX_EINVAL, "slab has more than 2^31-1 voxels");
        // the slab's box: global planes z0-1 .. z1 (planes outside the global box are void)
        std::vector<uint8_t> m((size_t)(nxy * ns), 0);
        std::vector<double> f(fibre ? (size_t)(3 * nxy * ns) : 0, 0.0);
        for (int zs = 0; zs < ns; zs++) {
            const int zg = z0 - 1 + zs;
            if (zg < 0 || zg >= nz) continue;
            memcpy(&m[zs * nxy], mask + zg * nxy, (size_t)nxy);
            if (fibre) memcpy(&f[3 * zs * nxy], fibre + 3 * zg * nxy, (size_t)(3 * nxy) * sizeof(double));
        }
        bbx_grid *g = nullptr;
        int rc = grid_create_common(nx, ny, ns, h, m.data(), fibre ? f.data() : nullptr, D_par,
                                    D_perp, precision, hip_stream, 1, L + 1, &g);
        if (rc) return rc;
        g->slab = 1;
        g->zoff = z0 - 1;
        const std::vector<int32_t> lists[4] = {plane_tissue(g, m.data(), 1), plane_tissue(g, m.data(), L),
                                               plane_tissue(g, m.data(), 0), plane_tissue(g, m.data(), L + 1)};
        int32_t **dst[4] = {&g->d_send[0], &g->d_send[1], &g->d_recv[0], &g->d_recv[1]};
        int64_t *cnt[4] = {&g->send_n[0], &g->send_n[1], &g->recv_n[0], &g->recv_n[1]};
        for (int k = 0; k < 4; k++) {
            *cnt[k] = (int64_t)lists[k].size();
            hipError_t e = dalloc(g, dst[k], lists[k].size() * sizeof(int32_t));
            if (e == hipSuccess && !lists[k].empty())
                e = hipMemcpy(*dst[k], lists[k].data(), lists[k].size() * sizeof(int32_t), hipMemcpyHostToDevice);
            if (e != hipSuccess) {
                std::string keep = hipGetErrorString(e);
                bbx_grid_destroy(g);
                return fail(BBX_ENOMEM, "halo lists: %s", keep.c_str());
            }
        }
        *out = g;
        return BBX_OK;
    } catch (...) {
        return fail(BBX_ENOMEM, "host allocation failed");
    }
}

int bbx_halo_pack(bbx_grid *g, int side, void *buf_dev, int64_t count)
{
    g_err.clear();
    if (!g) return fail(BBX_EINVAL, "grid is NULL");
    if (!g->slab) return fail(BBX_ESTATE, "not a slab grid (bbx_slab_create)");
    if (side != 0 && side != 1) return fail(BBX_EINVAL, "side must be 0 (lower) or 1 (upper)");
    if (count != g->send_n[side])
        return fail(BBX_EINVAL, "side %d sends %lld values, got count %lld", side,
                    (long long)g->send_n[side], (long long)count);
    if (count > 0 && !buf_dev) return fail(BBX_EINVAL, "buffer is NULL");
    hipError_t e = g->prec ? launch_gather<double>((const double *)g->d_V[g->cur], g->d_send[side], 0,
                                                   count, (double *)buf_dev, g->stream)
                           : launch_gather<float>((const float *)g->d_V[g->cur], g->d_send[side], 0,
                                                  count, (float *)buf_dev, g->stream);
    if (e != hipSuccess) return hip_fail(e, "halo pack");
    return BBX_OK;
}

int bbx_halo_unpack(bbx_grid *g, int side, const void *buf_dev, int64_t count)
{
    g_err.clear();
    if (!g) return fail(BBX_EINVAL, "grid is NULL");
    if (!g->slab) return fail(BBX_ESTATE, "not a slab grid (bbx_slab_create)");
    if (side != 0 && side != 1) return fail(BBX_EINVAL, "side must be 0 (lower) or 1 (upper)");
    if (count != g->recv_n[side])
        return fail(BBX_EINVAL, "side %d receives %lld values, got count %lld", side,
                    (long long)g->recv_n[side], (long long)count);
    if (count > 0 && !buf_dev) return fail(BBX_EINVAL, "buffer is NULL");
    hipError_t e = g->prec ? launch_scatter<double>((const double *)buf_dev, g->d_recv[side], count,
                                                    (double *)g->d_V[g->cur], g->stream)
                           : launch_scatter<float>((const float *)buf_dev, g->d_recv[side], count,
                                                   (float *)g->d_V[g->cur], g->stream);
    if (e != hipSuccess) return hip_fail(e, "halo unpack");
    return BBX_OK;
}

int bbx_model_set(bbx_grid *g, int model, const double *params, int nparams, double dt, int scheme)
{
    try {
        g_err.clear();
        if (!g) return fail(BBX_EINVAL, "grid is NULL");
        const int nv = model_nvar(model), np = model_nparams(model);
        if (nv < 0) return fail(BBX_EINVAL, "unknown model %d", model);
        if (nparams != np) return fail(BBX_EINVAL, "model %d takes %d parameters, got %d", model, np, nparams);
        if (np > 0 && !params) return fail(BBX_EINVAL, "params is NULL");
        for (int i = 0; i < np; i++)
            if (!isfinite(params[i])) return fail(BBX_EINVAL, "parameter %d is not finite", i);
        if (!(dt > 0) || !isfinite(dt)) return fail(BBX_EINVAL, "dt must be positive");
        if (scheme != BBX_SCHEME_ADDITIVE && scheme != BBX_SCHEME_SPLIT) return fail(BBX_EINVAL, "bad scheme");
        if (g->wsum_max > 0 && dt > 2.0 / g->wsum_max)
            return fail(BBX_EUNSTABLE, "dt %g exceeds the explicit diffusion bound %g", dt, 2.0 / g->wsum_max);
        int rc = g->prec ? alloc_state<double>(g, nv) : alloc_state<float>(g, nv);
        if (rc) return rc;
        g->model = model;
        g->nvar = nv;
        g->dt = dt;
        g->scheme = scheme;
        for (int i = 0; i < kMaxParams; i++) g->prm[i] = i < np ? params[i] : 0.0;
        g->n = 0;
        graph_drop(g);
        log_line("grid %p: model %d (%d variables), dt %g ms, %s scheme", (void *)g, model, nv, dt,
                 scheme == BBX_SCHEME_SPLIT ? "split" : "additive");
        return build_table(g);
    } catch (...) {
        return fail(BBX_ENOMEM, "host allocation failed");
    }
}

int bbx_state_set(bbx_grid *g, int var, const double *box_values)
{
    try {
        g_err.clear();
        if (!g) return fail(BBX_EINVAL, "grid is NULL");
        if (!box_values) return fail(BBX_EINVAL, "values is NULL");
        if (var < 0 || var >= g->nvar) return fail(BBX_EINVAL, "var %d out of range (nvar %d)", var, g->nvar);
        if (var > 0 && g->model < 0) return fail(BBX_ESTATE, "set a model first");
        return g->prec ? state_set_impl<double>(g, var, box_values) : state_set_impl<float>(g, var, box_values);
    } catch (...) {
        return fail(BBX_ENOMEM, "host allocation failed");
    }
}

int bbx_state_fill(bbx_grid *g, int var, double value)
{
    try {
        g_err.clear();
        if (!g) return fail(BBX_EINVAL, "grid is NULL");
        if (var < 0 || var >= g->nvar) return fail(BBX_EINVAL, "var %d out of range (nvar %d)", var, g->nvar);
        if (var > 0 && g->model < 0) return fail(BBX_ESTATE, "set a model first");
        if (!isfinite(value)) return fail(BBX_EINVAL, "value is not finite");
        return g->prec ? state_fill_impl<double>(g, var, value) : state_fill_impl<float>(g, var, value);
    } catch (...) {
        return fail(BBX_ENOMEM, "host allocation failed");
    }
}

int bbx_stimulus_add(bbx_grid *g, const uint8_t *region, double amplitude, double t_start,
                     double duration, double period, int count)
{
    try {
        g_err.clear();
        if (!g) return fail(BBX_EINVAL, "grid is NULL");
        if (!region) return fail(BBX_EINVAL, "region is NULL");
        if (!isfinite(amplitude) || !isfinite(t_start) || !isfinite(duration) || !isfinite(period))
            return fail(BBX_EINVAL, "stimulus numbers must be finite");
        if (t_start < 0 || duration < 0) return fail(BBX_EINVAL, "t_start and duration must be >= 0");
        if ((int)g->stims.size() >= kMaxStim) return fail(BBX_EINVAL, "at most %d stimuli", kMaxStim);
        std::vector<int32_t> h_idx;
        int rc = download_idx(g, h_idx);
        if (rc) return rc;
        const int k = (int)g->stims.size();
        std::vector<uint32_t> bits = g->h_stimbits;
        for (int64_t t = 0; t < g->nact; t++)
            if (region[g->dense ? t : h_idx[t]]) bits[t] |= 1u << k;
        if (!g->d_stimbits) {
            hipError_t e = dalloc(g, &g->d_stimbits, g->nact * sizeof(uint32_t));
            if (e != hipSuccess) return hip_fail(e, "hipMalloc");
        }
        if (g->nact)
            HIP_TRY(hipMemcpy(g->d_stimbits, bits.data(), g->nact * sizeof(uint32_t), hipMemcpyHostToDevice), "hipMemcpy");
        if (g->prec) {
            double a = amplitude;
            HIP_TRY(hipMemcpy((double *)g->d_stimamp + k, &a, sizeof a, hipMemcpyHostToDevice), "hipMemcpy");
        } else {
            float a = (float)amplitude;
            HIP_TRY(hipMemcpy((float *)g->d_stimamp + k, &a, sizeof a, hipMemcpyHostToDevice), "hipMemcpy");
        }
        g->h_stimbits.swap(bits);
        g->stims.push_back({amplitude, t_start, duration, period, count});
        graph_drop(g);
        return BBX_OK;
    } catch (...) {
        return fail(BBX_ENOMEM, "host allocation failed");
    }
}

int bbx_stimulus_clear(bbx_grid *g)
{
    g_err.clear();
    if (!g) return fail(BBX_EINVAL, "grid is NULL");
    g->stims.clear();
    graph_drop(g);
    std::fill(g->h_stimbits.begin(), g->h_stimbits.end(), 0u);
    if (g->d_stimbits && g->nact)
        HIP_TRY(hipMemset(g->d_stimbits, 0, g->nact * sizeof(uint32_t)), "hipMemset");
    return BBX_OK;
}

int bbx_recording_set(bbx_grid *g, double theta)
{
    try {
        g_err.clear();
        if (!g) return fail(BBX_EINVAL, "grid is NULL");
        graph_drop(g);
        if (isnan(theta)) { g->rec = 0; return BBX_OK; }
        if (!isfinite(theta)) return fail(BBX_EINVAL, "theta must be finite or NaN");
        return g->prec ? recording_impl<double>(g, theta) : recording_impl<float>(g, theta);
    } catch (...) {
        return fail(BBX_ENOMEM, "host allocation failed");
    }
}

int bbx_nan_check_set(bbx_grid *g, int64_t every)
{
    g_err.clear();
    if (!g) return fail(BBX_EINVAL, "grid is NULL");
    if (every < 0) return fail(BBX_EINVAL, "every must be >= 0");
    g->nan_every = every;
    return BBX_OK;
}

int bbx_ecg_set(bbx_grid *g, int nelec, const double *xyz_mm, int64_t every, int64_t max_samples)
{
    try {
        g_err.clear();
        if (!g) return fail(BBX_EINVAL, "grid is NULL");
        if (nelec < 0 || nelec > kMaxElectrodes) return fail(BBX_EINVAL, "nelec must be 0..%d", kMaxElectrodes);
        if (nelec > 0 && !xyz_mm) return fail(BBX_EINVAL, "xyz is NULL");
        if (nelec > 0 && (every < 0 || max_samples < 0 || max_samples > ((int64_t)1 << 26)))
            return fail(BBX_EINVAL, "every must be >= 0 and max_samples in 0..2^26");
        if (nelec > 0 && every > 0 && max_samples == 0) return fail(BBX_EINVAL, "sampling needs max_samples > 0");
        EcgElectrodes el = {};
        el.n = nelec;
        el.h = g->h;
        std::vector<uint8_t> mask;
        for (int e = 0; e < nelec; e++) {
            const double x = xyz_mm[3 * e], y = xyz_mm[3 * e + 1], z = xyz_mm[3 * e + 2];
            if (!isfinite(x) || !isfinite(y) || !isfinite(z)) return fail(BBX_EINVAL, "electrode %d not finite", e);
            // an electrode on a tissue voxel centre would divide by zero
            const double fx = x / g->h, fy = y / g->h, fz = z / g->h - g->zoff;
            if (fx == floor(fx) && fy == floor(fy) && fz == floor(fz) && fx >= 0 && fy >= 0 && fz >= 0 &&
                fx < g->nx && fy < g->ny && fz < g->nz) {
                if (mask.empty()) {
                    int rc = download_mask(g, mask);
                    if (rc) return rc;
                }
                if (mask[(size_t)fx + (size_t)g->nx * ((size_t)fy + (size_t)g->ny * (size_t)fz)])
                    return fail(BBX_EINVAL, "electrode %d sits on a tissue voxel centre", e);
            }
            el.x[e] = x;
            el.y[e] = y;
            el.z[e] = z - g->zoff * g->h;   // a slab's box starts at global plane zoff
        }
        HIP_TRY(hipStreamSynchronize(g->stream), "hipStreamSynchronize");
        dfree(g->d_ecg_series);
        g->d_ecg_series = nullptr;
        g->ecg_count = 0;
        g->ecg_every = 0;
        g->ecg_max = 0;
        g->ecg = el;
        if (nelec == 0) return BBX_OK;
        hipError_t e = hipSuccess;
        if (!g->d_ecg_parts) e = dalloc(g, &g->d_ecg_parts, (size_t)kEcgPartials * kMaxElectrodes * sizeof(double));
        if (e == hipSuccess && !g->d_ecg_now) e = dalloc(g, &g->d_ecg_now, kMaxElectrodes * sizeof(double));
        if (e == hipSuccess && every > 0)
            e = dalloc(g, &g->d_ecg_series, (size_t)max_samples * nelec * sizeof(double));
        if (e != hipSuccess) {
            g->ecg.n = 0;
            return hip_fail(e, "hipMalloc");
        }
        g->ecg_every = every;
        g->ecg_max = every > 0 ? max_samples : 0;
        return BBX_OK;
    } catch (...) {
        return fail(BBX_ENOMEM, "host allocation failed");
    }
}

int bbx_tabulation_set(bbx_grid *g, double dv)
{
    g_err.clear();
    if (!g) return fail(BBX_EINVAL, "grid is NULL");
    if (!(dv >= 0) || !isfinite(dv)) return fail(BBX_EINVAL, "dv must be >= 0");
    if (dv > 0) {
        if (g->prec != BBX_FP32) return fail(BBX_ENOTSUP, "tabulation is an FP32 variant");
        if (g->model != BBX_MODEL_CRN) return fail(BBX_ENOTSUP, "tabulation is provided for the CRN model");
        if (dv < 1e-4 || (kTabVmax - kTabVmin) / dv > 1e7) return fail(BBX_EINVAL, "dv out of range");
    }
    g->tab_dv = dv;
    graph_drop(g);
    return build_table(g);
}

int bbx_integrator_set(bbx_grid *g, int integrator)
{
    g_err.clear();
    if (!g) return fail(BBX_EINVAL, "grid is NULL");
    if (integrator != BBX_INTEGRATOR_EULER_RL && integrator != BBX_INTEGRATOR_RK4)
        return fail(BBX_EINVAL, "unknown integrator %d", integrator);
    if (integrator == BBX_INTEGRATOR_RK4 && g->sur)
        return fail(BBX_ENOTSUP, "the surrogate stands in for the Euler / Rush-Larsen step");
    g->integrator = integrator;
    graph_drop(g);
    return BBX_OK;
}

int bbx_graph_set(bbx_grid *g, int chunk)
{
    g_err.clear();
    if (!g) return fail(BBX_EINVAL, "grid is NULL");
    if (chunk < 0 || chunk > 4096 || (chunk & 1)) return fail(BBX_EINVAL, "chunk must be even, 0..4096");
    if (chunk > 0 && !g->stream) return fail(BBX_ENOTSUP, "graph capture needs a stream other than the null stream");
    graph_drop(g);
    g->chunk = chunk;
    return BBX_OK;
}

int bbx_clock_set(bbx_grid *g, int64_t step)
{
    g_err.clear();
    if (!g) return fail(BBX_EINVAL, "grid is NULL");
    if (step < 0) return fail(BBX_EINVAL, "step must be >= 0");
    g->n = step;
    return BBX_OK;
}

int bbx_step(bbx_grid *g, int64_t nsteps)
{
    try {
        g_err.clear();
        if (!g) return fail(BBX_EINVAL, "grid is NULL");
        if (nsteps < 0) return fail(BBX_EINVAL, "nsteps must be >= 0");
        if (g->model < 0) return fail(BBX_ESTATE, "set a model first");
        return g->prec ? step_impl<double>(g, nsteps) : step_impl<float>(g, nsteps);
    } catch (...) {
        return fail(BBX_ENOMEM, "host allocation failed");
    }
}

int bbx_readout(bbx_grid *g, int what, int var, const uint8_t *region, void *out, size_t out_bytes,
                int out_on_device)
{
    try {
        g_err.clear();
        if (!g) return fail(BBX_EINVAL, "grid is NULL");
        if (!out) return fail(BBX_EINVAL, "out is NULL");
        return g->prec ? readout_impl<double>(g, what, var, region, out, out_bytes, out_on_device)
                       : readout_impl<float>(g, what, var, region, out, out_bytes, out_on_device);
    } catch (...) {
        return fail(BBX_ENOMEM, "host allocation failed");
    }
}

}  // extern "C"

namespace {

template <typename T>
int tips_impl(bbx_grid *g, int vu, double ul, int vv, double vl, double *stats, double *points,
              int64_t max_points, int64_t *npoints)
{
    if (!g->dense && !g->d_map) {
        hipError_t e = dalloc(g, &g->d_map, (size_t)g->nbox * sizeof(int32_t));
        if (e != hipSuccess) return hip_fail(e, "hipMalloc");
        e = launch_box_map(g->d_map, g->nbox, g->d_idx, g->nact, g->stream);
        if (e != hipSuccess) {
            dfree(g->d_map);
            g->d_map = nullptr;
            return hip_fail(e, "box map");
        }
    }
    const int64_t cap = points ? max_points : 0;
    DevBuf part, pts;
    HIP_TRY(hipMalloc(&part.p, kTipPartBytes + 8 * sizeof(double) + sizeof(unsigned long long)), "hipMalloc");
    if (cap > 0) HIP_TRY(hipMalloc(&pts.p, (size_t)cap * 3 * sizeof(double)), "hipMalloc");
    double *out = (double *)((char *)part.p + kTipPartBytes);
    unsigned long long *cnt = (unsigned long long *)(out + 8);
    HIP_TRY(launch_fill<int>((int *)cnt, 0, 2, g->stream), "fill");
    TipLaunch<T> L = {};
    L.nx = g->nx; L.ny = g->ny; L.nz = g->nz; L.dense = g->dense;
    // a slab searches its own planes only (its halo planes are its neighbours' own) and
    // reports global coordinates
    L.z0 = g->slab ? 1 : 0;
    L.z1 = g->slab ? g->nz - 1 : g->nz;
    L.zoff = g->slab ? g->zoff : 0;
    L.h = g->h; L.ul = ul; L.vl = vl;
    L.map = g->d_map;
    const T *V = (const T *)g->d_V[g->cur], *st = (const T *)g->d_st;
    if (vu == 0) L.u_box = V; else L.u_list = st + (int64_t)(vu - 1) * g->pitch;
    if (vv == 0) L.v_box = V; else L.v_list = st + (int64_t)(vv - 1) * g->pitch;
    L.part = (double *)part.p;
    L.out = out;
    L.pts = (double *)pts.p;
    L.max_pts = cap;
    L.count = cnt;
    if (g->nx >= 2 && g->ny >= 2 && g->nact > 0 && L.z1 > L.z0) {
        HIP_TRY(launch_tips<T>(L, g->stream), "tips");
    } else {
        HIP_TRY(launch_fill<double>(out, 0.0, 7, g->stream), "fill");
    }
    double sums[7];
    unsigned long long n = 0;
    HIP_TRY(hipMemcpyAsync(sums, out, sizeof sums, hipMemcpyDeviceToHost, g->stream), "hipMemcpyAsync");
    HIP_TRY(hipMemcpyAsync(&n, cnt, sizeof n, hipMemcpyDeviceToHost, g->stream), "hipMemcpyAsync");
    HIP_TRY(hipStreamSynchronize(g->stream), "hipStreamSynchronize");
    const int64_t nw = (int64_t)n < cap ? (int64_t)n : cap;
    if (nw > 0) {
        HIP_TRY(hipMemcpyAsync(points, pts.p, (size_t)nw * 3 * sizeof(double), hipMemcpyDeviceToHost,
                               g->stream), "hipMemcpyAsync");
        HIP_TRY(hipStreamSynchronize(g->stream), "hipStreamSynchronize");
    }
    stats[0] = sums[0];
    for (int i = 1; i < 7; i++) stats[i] = 0.0;
    if (sums[0] > 0) {
        for (int i = 0; i < 3; i++) {
            const double mean = sums[1 + i] / sums[0];
            stats[1 + i] = mean;
            stats[4 + i] = sqrt(fmax(sums[4 + i] / sums[0] - mean * mean, 0.0));
        }
    }
    if (npoints) *npoints = (int64_t)n;
    return BBX_OK;
}

}  // namespace

extern "C" {

int bbx_tips(bbx_grid *g, int var_u, double u_level, int var_v, double v_level, double *stats,
             double *points, int64_t max_points, int64_t *npoints)
{
    try {
        g_err.clear();
        if (!g || !stats) return fail(BBX_EINVAL, "NULL argument");
        if (g->model < 0) return fail(BBX_ESTATE, "set a model first");
        if (var_u < 0 || var_u >= g->nvar || var_v < 0 || var_v >= g->nvar)
            return fail(BBX_EINVAL, "variables must be in [0, %d)", g->nvar);
        if (!isfinite(u_level) || !isfinite(v_level)) return fail(BBX_EINVAL, "levels must be finite");
        if (max_points < 0 || max_points > ((int64_t)1 << 28)) return fail(BBX_EINVAL, "max_points out of range");
        return g->prec ? tips_impl<double>(g, var_u, u_level, var_v, v_level, stats, points, max_points, npoints)
                       : tips_impl<float>(g, var_u, u_level, var_v, v_level, stats, points, max_points, npoints);
    } catch (...) {
        return fail(BBX_ENOMEM, "host allocation failed");
    }
}

int bbx_info(const bbx_grid *g, int what, int64_t *out)
{
    g_err.clear();
    if (!g || !out) return fail(BBX_EINVAL, "NULL argument");
    switch (what) {
    case BBX_INFO_NACTIVE: *out = g->nact; return BBX_OK;
    case BBX_INFO_NVAR: *out = g->nvar; return BBX_OK;
    case BBX_INFO_NBOX: *out = g->nbox; return BBX_OK;
    case BBX_INFO_DEVICE_BYTES: *out = (int64_t)g->bytes; return BBX_OK;
    case BBX_INFO_SEND_LO: *out = g->send_n[0]; return BBX_OK;
    case BBX_INFO_SEND_HI: *out = g->send_n[1]; return BBX_OK;
    case BBX_INFO_RECV_LO: *out = g->recv_n[0]; return BBX_OK;
    case BBX_INFO_RECV_HI: *out = g->recv_n[1]; return BBX_OK;
    default: return fail(BBX_EINVAL, "unknown info %d", what);
    }
}

void bbx_grid_destroy(bbx_grid *g)
{
    if (!g) return;
    (void)hipStreamSynchronize(g->stream);
    free_all(g);
    delete g;
}

}  // extern "C"

// ============================================================================ surrogate network

struct bbx_mlp {
    int nin = 0, nout = 0, np = 0;
    hipStream_t stream = nullptr;
    float *d_p = nullptr, *d_g = nullptr, *d_m = nullptr, *d_v = nullptr;
    double *d_loss = nullptr, *d_stats = nullptr;
    int64_t t = 0;           // Adam steps taken
    MlpDev dev = {};
    MlpScratch w = {};
    int64_t cap = 0;         // batch capacity of the scratch (rounded to 32)
    std::vector<void *> bufs;
};

namespace {

hipError_t mlp_alloc(bbx_mlp *m, void **p, size_t bytes)
{
    hipError_t e = hipMalloc(p, bytes ? bytes : 1);
    if (e == hipSuccess) m->bufs.push_back(*p);
    return e;
}

void mlp_free(bbx_mlp *m)
{
    for (void *p : m->bufs) (void)hipFree(p);
    m->bufs.clear();
}

int mlp_scratch(bbx_mlp *m, int64_t B)
{
    const int64_t Bp = (B + 31) / 32 * 32;
    if (Bp <= m->cap) return BBX_OK;
    void *ps[] = {m->w.xb, m->w.tt, m->w.xf, m->w.h1, m->w.h2, m->w.dz1, m->w.dz2, m->w.dO, m->w.part};
    for (void *p : ps) {
        if (!p) continue;
        for (size_t i = 0; i < m->bufs.size(); i++)
            if (m->bufs[i] == p) { (void)hipFree(p); m->bufs.erase(m->bufs.begin() + i); break; }
    }
    m->w = MlpScratch{};
    m->cap = 0;
    hipError_t e;
    const size_t bf = sizeof(__bf16);
    if ((e = mlp_alloc(m, (void **)&m->w.xb, Bp * kP * bf)) != hipSuccess) return hip_fail(e, "hipMalloc");
    if ((e = mlp_alloc(m, (void **)&m->w.tt, Bp * kP * sizeof(float))) != hipSuccess) return hip_fail(e, "hipMalloc");
    if ((e = mlp_alloc(m, (void **)&m->w.xf, Bp * kP * bf)) != hipSuccess) return hip_fail(e, "hipMalloc");
    if ((e = mlp_alloc(m, (void **)&m->w.dO, Bp * kP * bf)) != hipSuccess) return hip_fail(e, "hipMalloc");
    __bf16 **hs[] = {&m->w.h1, &m->w.h2, &m->w.dz1, &m->w.dz2};
    for (__bf16 **h : hs)
        if ((e = mlp_alloc(m, (void **)h, Bp * kH * bf)) != hipSuccess) return hip_fail(e, "hipMalloc");
    if ((e = mlp_alloc(m, (void **)&m->w.part, (Bp / 16) * kPart * sizeof(float))) != hipSuccess)
        return hip_fail(e, "hipMalloc");
    m->cap = Bp;
    return BBX_OK;
}

}  // namespace

extern "C" {

int bbx_mlp_create(int nin, int nout, uint64_t seed, void *hip_stream, bbx_mlp **out)
{
    try {
        g_err.clear();
        if (!out) return fail(BBX_EINVAL, "out is NULL");
        *out = nullptr;
        if (nin < 1 || nin > kP || nout < 1 || nout > kP)
            return fail(BBX_EINVAL, "nin and nout must be in [1, %d]", kP);
        int ndev = 0;
        if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return fail(BBX_EDEVICE, "no HIP device");
        bbx_mlp *m = new bbx_mlp();
        m->nin = nin;
        m->nout = nout;
        m->np = mlp_nparams(nin, nout);
        m->stream = (hipStream_t)hip_stream;
        m->dev.nin = nin;
        m->dev.nout = nout;
        hipError_t e = hipSuccess;
        const size_t pb = (size_t)m->np * sizeof(float);
        float **fs[] = {&m->d_p, &m->d_g, &m->d_m, &m->d_v};
        for (float **f : fs)
            if (e == hipSuccess) e = mlp_alloc(m, (void **)f, pb);
        if (e == hipSuccess) e = mlp_alloc(m, (void **)&m->d_loss, sizeof(double));
        if (e == hipSuccess) e = mlp_alloc(m, (void **)&m->d_stats, 2 * kP * 4 * sizeof(double));
        if (e == hipSuccess) e = mlp_alloc(m, (void **)&m->dev.w1, kH * kS1 * sizeof(__bf16));
        if (e == hipSuccess) e = mlp_alloc(m, (void **)&m->dev.w3t, kH * kS1 * sizeof(__bf16));
        if (e == hipSuccess) e = mlp_alloc(m, (void **)&m->dev.w2, kH * kS2 * sizeof(__bf16));
        if (e == hipSuccess) e = mlp_alloc(m, (void **)&m->dev.w2t, kH * kS2 * sizeof(__bf16));
        if (e == hipSuccess) e = mlp_alloc(m, (void **)&m->dev.w3, kP * kS2 * sizeof(__bf16));
        if (e == hipSuccess) e = mlp_alloc(m, (void **)&m->dev.bias, (2 * kH + kP) * sizeof(float));
        if (e == hipSuccess) e = mlp_alloc(m, (void **)&m->dev.norm, 4 * kP * sizeof(float));
        if (e != hipSuccess) {
            mlp_free(m);
            delete m;
            return hip_fail(e, "hipMalloc");
        }
        float norm[4 * kP];
        for (int i = 0; i < kP; i++) {
            norm[i] = 0.f;
            norm[kP + i] = 1.f;
            norm[2 * kP + i] = 0.f;
            norm[3 * kP + i] = 1.f;
        }
        hipStream_t st = m->stream;
        if ((e = hipMemcpyAsync(m->dev.norm, norm, sizeof norm, hipMemcpyHostToDevice, st)) == hipSuccess &&
            (e = hipMemsetAsync(m->d_m, 0, pb, st)) == hipSuccess &&
            (e = hipMemsetAsync(m->d_v, 0, pb, st)) == hipSuccess &&
            (e = hipMemsetAsync(m->d_g, 0, pb, st)) == hipSuccess &&
            (e = mlp_init(m->d_p, nin, nout, seed, st)) == hipSuccess &&
            (e = mlp_pack(m->d_p, m->dev, st)) == hipSuccess)
            e = hipStreamSynchronize(st);
        if (e != hipSuccess) {
            mlp_free(m);
            delete m;
            return hip_fail(e, "network initialisation");
        }
        *out = m;
        return BBX_OK;
    } catch (...) {
        return fail(BBX_ENOMEM, "host allocation failed");
    }
}

int bbx_mlp_params(bbx_mlp *m, int set, float *host, size_t count)
{
    g_err.clear();
    if (!m || !host) return fail(BBX_EINVAL, "NULL argument");
    if (count != (size_t)m->np) return fail(BBX_EINVAL, "the network has %d parameters", m->np);
    if (set) {
        for (size_t i = 0; i < count; i++)
            if (!isfinite(host[i])) return fail(BBX_EINVAL, "parameter %zu is not finite", i);
        HIP_TRY(hipMemcpyAsync(m->d_p, host, count * sizeof(float), hipMemcpyHostToDevice, m->stream), "hipMemcpyAsync");
        HIP_TRY(mlp_pack(m->d_p, m->dev, m->stream), "pack");
    } else {
        HIP_TRY(hipMemcpyAsync(host, m->d_p, count * sizeof(float), hipMemcpyDeviceToHost, m->stream), "hipMemcpyAsync");
    }
    HIP_TRY(hipStreamSynchronize(m->stream), "hipStreamSynchronize");
    return BBX_OK;
}

int bbx_mlp_norm(bbx_mlp *m, int set, float *host)
{
    g_err.clear();
    if (!m || !host) return fail(BBX_EINVAL, "NULL argument");
    if (set) {
        for (int i = 0; i < 4 * kP; i++)
            if (!isfinite(host[i])) return fail(BBX_EINVAL, "normalisation entry %d is not finite", i);
        for (int i = 0; i < kP; i++)
            if (host[3 * kP + i] < 0.f) return fail(BBX_EINVAL, "out_sigma %d is negative", i);
        HIP_TRY(hipMemcpyAsync(m->dev.norm, host, 4 * kP * sizeof(float), hipMemcpyHostToDevice, m->stream), "hipMemcpyAsync");
    } else {
        HIP_TRY(hipMemcpyAsync(host, m->dev.norm, 4 * kP * sizeof(float), hipMemcpyDeviceToHost, m->stream), "hipMemcpyAsync");
    }
    HIP_TRY(hipStreamSynchronize(m->stream), "hipStreamSynchronize");
    return BBX_OK;
}

int bbx_mlp_fit_norm(bbx_mlp *m, const float *S_dev, const float *S1_dev, int64_t n, double *stats)
{
    try {
        g_err.clear();
        if (!m || !S_dev || !S1_dev) return fail(BBX_EINVAL, "NULL argument");
        if (m->nin != m->nout) return fail(BBX_EINVAL, "fitting needs nin == nout");
        if (n < 2) return fail(BBX_EINVAL, "need at least 2 samples");
        HIP_TRY(mlp_stats(S_dev, S1_dev, n, m->nin, m->d_stats, m->stream), "stats");
        std::vector<double> st(2 * kP * 4);
        HIP_TRY(hipMemcpyAsync(st.data(), m->d_stats, st.size() * sizeof(double), hipMemcpyDeviceToHost, m->stream), "hipMemcpyAsync");
        HIP_TRY(hipStreamSynchronize(m->stream), "hipStreamSynchronize");
        float norm[4 * kP];
        for (int i = 0; i < kP; i++) {
            const double mi = st[i * 4], si = st[i * 4 + 1];
            const double mo = st[(kP + i) * 4], so = st[(kP + i) * 4 + 1];
            norm[i] = (float)mi;
            norm[kP + i] = (float)(si > 0 ? 1.0 / si : 1.0);
            norm[2 * kP + i] = (float)mo;
            norm[3 * kP + i] = (float)so;   // 0: a constant increment, predicted exactly
        }
        HIP_TRY(hipMemcpyAsync(m->dev.norm, norm, sizeof norm, hipMemcpyHostToDevice, m->stream), "hipMemcpyAsync");
        HIP_TRY(hipStreamSynchronize(m->stream), "hipStreamSynchronize");
        if (stats) {
            for (int i = 0; i < kP; i++) {
                stats[0 * kP + i] = st[i * 4];
                stats[1 * kP + i] = st[i * 4 + 1];
                stats[2 * kP + i] = st[i * 4 + 2];
                stats[3 * kP + i] = st[i * 4 + 3];
                stats[4 * kP + i] = st[(kP + i) * 4];
                stats[5 * kP + i] = st[(kP + i) * 4 + 1];
                stats[6 * kP + i] = fmax(fabs(st[(kP + i) * 4 + 2]), fabs(st[(kP + i) * 4 + 3]));
            }
        }
        return BBX_OK;
    } catch (...) {
        return fail(BBX_ENOMEM, "host allocation failed");
    }
}

int bbx_mlp_forward(bbx_mlp *m, const float *X_dev, int64_t n, float *Y_dev)
{
    g_err.clear();
    if (!m || !X_dev || !Y_dev) return fail(BBX_EINVAL, "NULL argument");
    if (n < 0) return fail(BBX_EINVAL, "n must be >= 0");
    HIP_TRY(mlp_forward(m->dev, X_dev, n, Y_dev, m->stream), "forward");
    return BBX_OK;
}

int bbx_mlp_grad(bbx_mlp *m, const float *X_dev, const float *T_dev, int64_t n, float *grad_host,
                 double *loss)
{
    try {
        g_err.clear();
        if (!m || !X_dev || !T_dev) return fail(BBX_EINVAL, "NULL argument");
        if (n < 1 || n > kMaxBatch) return fail(BBX_EINVAL, "n must be in [1, %lld]", (long long)kMaxBatch);
        int rc = mlp_scratch(m, n);
        if (rc) return rc;
        HIP_TRY(mlp_grad(m->dev, m->w, 0, X_dev, T_dev, n, n, 0, 0, m->d_g, m->d_loss, m->stream), "gradient");
        if (grad_host)
            HIP_TRY(hipMemcpyAsync(grad_host, m->d_g, m->np * sizeof(float), hipMemcpyDeviceToHost, m->stream), "hipMemcpyAsync");
        if (loss) HIP_TRY(hipMemcpyAsync(loss, m->d_loss, sizeof(double), hipMemcpyDeviceToHost, m->stream), "hipMemcpyAsync");
        HIP_TRY(hipStreamSynchronize(m->stream), "hipStreamSynchronize");
        return BBX_OK;
    } catch (...) {
        return fail(BBX_ENOMEM, "host allocation failed");
    }
}

int bbx_mlp_adam(bbx_mlp *m, float lr, float beta1, float beta2, float eps)
{
    g_err.clear();
    if (!m) return fail(BBX_EINVAL, "NULL argument");
    if (!(lr > 0) || !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps > 0))
        return fail(BBX_EINVAL, "bad Adam hyper-parameters");
    m->t += 1;
    HIP_TRY(mlp_adam(m->d_p, m->d_m, m->d_v, m->d_g, m->np, lr, beta1, beta2, eps, m->t, m->stream), "adam");
    HIP_TRY(mlp_pack(m->d_p, m->dev, m->stream), "pack");
    return BBX_OK;
}

int bbx_mlp_train(bbx_mlp *m, const float *S_dev, const float *S1_dev, int64_t n, int64_t batch,
                  int64_t iters, float lr, uint64_t seed, float *loss_hist)
{
    try {
        g_err.clear();
        if (!m || !S_dev || !S1_dev) return fail(BBX_EINVAL, "NULL argument");
        if (m->nin != m->nout) return fail(BBX_EINVAL, "training on state pairs needs nin == nout");
        if (n < 1 || batch < 1 || batch > kMaxBatch || iters < 0)
            return fail(BBX_EINVAL, "bad n / batch / iters");
        if (!(lr > 0)) return fail(BBX_EINVAL, "lr must be positive");
        int rc = mlp_scratch(m, batch);
        if (rc) return rc;
        DevBuf lh;
        if (loss_hist && iters > 0) HIP_TRY(hipMalloc(&lh.p, iters * sizeof(double)), "hipMalloc");
        for (int64_t it = 0; it < iters; it++) {
            double *ls = lh.p ? (double *)lh.p + it : m->d_loss;
            HIP_TRY(mlp_grad(m->dev, m->w, 1, S_dev, S1_dev, n, batch, seed, (uint64_t)it, m->d_g, ls,
                             m->stream), "gradient");
            m->t += 1;
            HIP_TRY(mlp_adam(m->d_p, m->d_m, m->d_v, m->d_g, m->np, lr, 0.9f, 0.999f, 1e-8f, m->t,
                             m->stream), "adam");
            HIP_TRY(mlp_pack(m->d_p, m->dev, m->stream), "pack");
        }
        if (lh.p) {
            std::vector<double> tmp((size_t)iters);
            HIP_TRY(hipMemcpyAsync(tmp.data(), lh.p, iters * sizeof(double), hipMemcpyDeviceToHost, m->stream), "hipMemcpyAsync");
            HIP_TRY(hipStreamSynchronize(m->stream), "hipStreamSynchronize");
            for (int64_t i = 0; i < iters; i++) loss_hist[i] = (float)tmp[(size_t)i];
        }
        HIP_TRY(hipStreamSynchronize(m->stream), "hipStreamSynchronize");
        return BBX_OK;
    } catch (...) {
        return fail(BBX_ENOMEM, "host allocation failed");
    }
}

int bbx_mlp_anchor(bbx_mlp *m, const float *s0_dev, const float *s1_dev)
{
    g_err.clear();
    if (!m || !s0_dev || !s1_dev) return fail(BBX_EINVAL, "NULL argument");
    if (m->nin != m->nout) return fail(BBX_EINVAL, "anchoring needs nin == nout");
    HIP_TRY(mlp_anchor(m->dev, s0_dev, s1_dev, m->d_p, m->stream), "anchor");
    HIP_TRY(hipStreamSynchronize(m->stream), "hipStreamSynchronize");
    return BBX_OK;
}

void bbx_mlp_destroy(bbx_mlp *m)
{
    if (!m) return;
    (void)hipStreamSynchronize(m->stream);
    mlp_free(m);
    delete m;
}

int bbx_sample_states(bbx_grid *g, int64_t n, uint64_t seed, float *out_dev)
{
    g_err.clear();
    if (!g || !out_dev) return fail(BBX_EINVAL, "NULL argument");
    if (g->prec != BBX_FP32) return fail(BBX_ENOTSUP, "state sampling needs an FP32 grid");
    if (g->model < 0) return fail(BBX_ESTATE, "set a model first");
    if (n < 0) return fail(BBX_EINVAL, "n must be >= 0");
    if (g->nact == 0 && n > 0) return fail(BBX_EINVAL, "the grid has no tissue");
    StepArgs<float> a = make_args<float>(g);
    a.Vin = (const float *)g->d_V[g->cur];
    HIP_TRY(launch_sample(a, g->nvar, n, seed, out_dev, g->stream), "sample");
    return BBX_OK;
}

int bbx_ionic_map(bbx_grid *g, const float *in_dev, int64_t n, float *out_dev)
{
    g_err.clear();
    if (!g || !in_dev || !out_dev) return fail(BBX_EINVAL, "NULL argument");
    if (g->prec != BBX_FP32) return fail(BBX_ENOTSUP, "the ionic map runs on FP32 grids");
    if (g->model < 0) return fail(BBX_ESTATE, "set a model first");
    if (n < 0) return fail(BBX_EINVAL, "n must be >= 0");
    StepArgs<float> a = make_args<float>(g);
    HIP_TRY(launch_ionic_map(g->model, a, g->nvar, in_dev, n, out_dev, g->stream), "ionic map");
    return BBX_OK;
}

}  // extern "C"

namespace {

// Validation shared by the two ways of attaching a surrogate.
int surrogate_check(const bbx_grid *g, int nin, int nout, const float *lo, const float *hi,
                    float dv_max)
{
    if (g->prec != BBX_FP32) return fail(BBX_ENOTSUP, "the surrogate runs on FP32 grids");
    if (g->integrator != BBX_INTEGRATOR_EULER_RL)
        return fail(BBX_ENOTSUP, "the surrogate stands in for the Euler / Rush-Larsen step");
    if (g->model != BBX_MODEL_BARKLEY && g->model != BBX_MODEL_FHN && g->model != BBX_MODEL_CRN &&
        g->model != BBX_MODEL_TP06)
        return fail(BBX_ENOTSUP, "no surrogate step for model %d", g->model);
    if (nin != g->nvar || nout != g->nvar)
        return fail(BBX_EINVAL, "network is %d -> %d, the model has %d variables", nin, nout, g->nvar);
    if (!lo || !hi) return fail(BBX_EINVAL, "lo / hi is NULL");
    if (!(dv_max >= 0)) return fail(BBX_EINVAL, "dv_max must be >= 0");
    return BBX_OK;
}

// Device buffers of the grid's network copy and its step lists (first attachment).
int surrogate_alloc(bbx_grid *g, int nin, int nout)
{
    if (g->sur_nblk) return BBX_OK;                 // set once every buffer below is in place
    hipError_t e;
    g->snet.nin = nin;
    g->snet.nout = nout;
    // one list segment per classifier workgroup (kBlock voxels)
    const int nb = (int)((g->nact + kBlock - 1) / kBlock);
    const size_t bytes0 = g->bytes;
    if ((e = dalloc(g, &g->snet.w1, kH * kS1 * sizeof(__bf16))) != hipSuccess ||
        (e = dalloc(g, &g->snet.w2, kH * kS2 * sizeof(__bf16))) != hipSuccess ||
        (e = dalloc(g, &g->snet.w3, kP * kS2 * sizeof(__bf16))) != hipSuccess ||
        (e = dalloc(g, &g->snet.bias, (2 * kH + kP) * sizeof(float))) != hipSuccess ||
        (e = dalloc(g, &g->snet.norm, 4 * kP * sizeof(float))) != hipSuccess ||
        (e = dalloc(g, &g->d_slo, kP * sizeof(float))) != hipSuccess ||
        (e = dalloc(g, &g->d_shi, kP * sizeof(float))) != hipSuccess ||
        (e = dalloc(g, &g->d_acc_list, (size_t)(nb ? nb : 1) * kBlock * sizeof(int32_t))) != hipSuccess ||
        (e = dalloc(g, &g->d_acc_cnt, (size_t)(nb ? nb : 1) * sizeof(int32_t))) != hipSuccess ||
        (e = dalloc(g, &g->d_fb, (size_t)(nb ? nb : 1) * sizeof(unsigned long long))) != hipSuccess) {
        // a failed attempt keeps nothing, so that a later one starts from scratch
        void **ps[] = {(void **)&g->snet.w1, (void **)&g->snet.w2, (void **)&g->snet.w3,
                       (void **)&g->snet.bias, (void **)&g->snet.norm, (void **)&g->d_slo,
                       (void **)&g->d_shi, (void **)&g->d_acc_list, (void **)&g->d_acc_cnt,
                       (void **)&g->d_fb};
        for (void **p : ps) {
            dfree(*p);
            *p = nullptr;
        }
        g->bytes = bytes0;
        return hip_fail(e, "hipMalloc");
    }
    g->sur_nblk = nb > 0 ? nb : 1;
    return BBX_OK;
}

// Box, counters and flags after the weights are in place.
int surrogate_finish(bbx_grid *g, const float *lo, const float *hi, float dv_max)
{
    hipStream_t st = g->stream;
    HIP_TRY(hipMemcpyAsync(g->d_slo, lo, g->nvar * sizeof(float), hipMemcpyHostToDevice, st), "copy");
    HIP_TRY(hipMemcpyAsync(g->d_shi, hi, g->nvar * sizeof(float), hipMemcpyHostToDevice, st), "copy");
    const int64_t nb = g->sur_nblk ? g->sur_nblk : 1;
    HIP_TRY(launch_fill<int>(g->d_acc_cnt, 0, nb, st), "fill");
    HIP_TRY(launch_fill<int>((int *)g->d_fb, 0, 2 * nb, st), "fill");
    HIP_TRY(hipStreamSynchronize(st), "hipStreamSynchronize");
    g->dv_max = dv_max;
    g->sur = 1;
    graph_drop(g);
    log_line("grid %p: surrogate attached (%d -> 128 -> 128 -> %d, |dV| <= %g mV per step)", (void *)g,
             g->snet.nin, g->snet.nout, dv_max);
    return BBX_OK;
}

}  // namespace

extern "C" {

int bbx_surrogate_import(bbx_grid *g, int nin, int nout, const uint16_t *weights_bf16,
                         const float *biases, const float *norm, const float *lo, const float *hi,
                         float dv_max)
{
    try {
        g_err.clear();
        if (!g) return fail(BBX_EINVAL, "grid is NULL");
        if (!weights_bf16 || !biases || !norm) return fail(BBX_EINVAL, "NULL argument");
        if (nin < 1 || nin > kP || nout < 1 || nout > kP)
            return fail(BBX_EINVAL, "nin and nout must be in [1, %d]", kP);
        int rc = surrogate_check(g, nin, nout, lo, hi, dv_max);
        if (rc) return rc;
        for (int i = 0; i < 4 * kP; i++)
            if (!isfinite(norm[i])) return fail(BBX_EINVAL, "normalisation entry %d is not finite", i);
        for (int i = 0; i < kP; i++)
            if (norm[3 * kP + i] < 0.f) return fail(BBX_EINVAL, "out_sigma %d is negative", i);
        // flat FP32 parameters W1 b1 W2 b2 W3 b3 from the BF16 weights (exact) and biases
        const int nw1 = kH * nin, nw2 = kH * kH, nw3 = nout * kH;
        std::vector<float> p((size_t)mlp_nparams(nin, nout));
        auto bf = [](uint16_t b) { uint32_t u = (uint32_t)b << 16; float f; memcpy(&f, &u, 4); return f; };
        size_t o = 0, w = 0, bo = 0;
        for (int i = 0; i < nw1; i++) p[o++] = bf(weights_bf16[w++]);
        for (int i = 0; i < kH; i++) p[o++] = biases[bo++];
        for (int i = 0; i < nw2; i++) p[o++] = bf(weights_bf16[w++]);
        for (int i = 0; i < kH; i++) p[o++] = biases[bo++];
        for (int i = 0; i < nw3; i++) p[o++] = bf(weights_bf16[w++]);
        for (int i = 0; i < nout; i++) p[o++] = biases[bo++];
        for (float v : p)
            if (!isfinite(v)) return fail(BBX_EINVAL, "a network parameter is not finite");
        rc = surrogate_alloc(g, nin, nout);
        if (rc) return rc;
        DevBuf dp;
        HIP_TRY(hipMalloc(&dp.p, p.size() * sizeof(float)), "hipMalloc");
        HIP_TRY(hipMemcpyAsync(dp.p, p.data(), p.size() * sizeof(float), hipMemcpyHostToDevice, g->stream),
                "hipMemcpyAsync");
        MlpDev d = g->snet;
        d.w2t = nullptr;
        d.w3t = nullptr;
        HIP_TRY(mlp_pack((const float *)dp.p, d, g->stream), "pack");
        HIP_TRY(hipMemcpyAsync(g->snet.norm, norm, 4 * kP * sizeof(float), hipMemcpyHostToDevice, g->stream),
                "hipMemcpyAsync");
        HIP_TRY(hipStreamSynchronize(g->stream), "hipStreamSynchronize");
        return surrogate_finish(g, lo, hi, dv_max);
    } catch (...) {
        return fail(BBX_ENOMEM, "host allocation failed");
    }
}

int bbx_surrogate_set(bbx_grid *g, const bbx_mlp *m, const float *lo, const float *hi, float dv_max)
{
    try {
        g_err.clear();
        if (!g) return fail(BBX_EINVAL, "grid is NULL");
        if (!m) {
            g->sur = 0;
            graph_drop(g);
            return BBX_OK;
        }
        int rc = surrogate_check(g, m->nin, m->nout, lo, hi, dv_max);
        if (rc) return rc;
        rc = surrogate_alloc(g, m->nin, m->nout);
        if (rc) return rc;
        hipStream_t st = g->stream;
        // the network's device copies are ordered on its own stream: finish them first
        HIP_TRY(hipStreamSynchronize(m->stream), "hipStreamSynchronize");
        HIP_TRY(hipMemcpyAsync(g->snet.w1, m->dev.w1, kH * kS1 * sizeof(__bf16), hipMemcpyDeviceToDevice, st), "copy");
        HIP_TRY(hipMemcpyAsync(g->snet.w2, m->dev.w2, kH * kS2 * sizeof(__bf16), hipMemcpyDeviceToDevice, st), "copy");
        HIP_TRY(hipMemcpyAsync(g->snet.w3, m->dev.w3, kP * kS2 * sizeof(__bf16), hipMemcpyDeviceToDevice, st), "copy");
        HIP_TRY(hipMemcpyAsync(g->snet.bias, m->dev.bias, (2 * kH + kP) * sizeof(float), hipMemcpyDeviceToDevice, st), "copy");
        HIP_TRY(hipMemcpyAsync(g->snet.norm, m->dev.norm, 4 * kP * sizeof(float), hipMemcpyDeviceToDevice, st), "copy");
        return surrogate_finish(g, lo, hi, dv_max);
    } catch (...) {
        return fail(BBX_ENOMEM, "host allocation failed");
    }
}

}  // extern "C"

// ============================================================================ allocation-free gradient
// bbx_mlp_grad_static: the gradient of bbx_mlp_grad for callers that cannot allocate
// device memory.  Its training scratch (batch inputs and targets, feature-major
// activations and deltas, per-tile partial sums) lives in one file-scope device array
// sized for kStaticBatch samples.  Host code never passes the array's name to a kernel
// (on the host it only names a stand-in): its device address is looked up once per
// device with hipGetSymbolAddress and kept in g_static_ptr.

namespace {

constexpr int64_t kStaticBatch = 4096;     // largest batch of bbx_mlp_grad_static
constexpr size_t kAl = 256;
constexpr size_t al(size_t b) { return (b + kAl - 1) / kAl * kAl; }
// carve of the scratch for kStaticBatch samples, in the order of MlpScratch
constexpr size_t kScrXb = al(kStaticBatch * kP * sizeof(__bf16));
constexpr size_t kScrTt = al(kStaticBatch * kP * sizeof(float));
constexpr size_t kScrXf = al(kStaticBatch * kP * sizeof(__bf16));
constexpr size_t kScrDo = al(kStaticBatch * kP * sizeof(__bf16));
constexpr size_t kScrH = al(kStaticBatch * kH * sizeof(__bf16));
constexpr size_t kScrPart = al(kStaticBatch / 16 * kPart * sizeof(float));
constexpr size_t kStaticBytes = kScrXb + kScrTt + kScrXf + kScrDo + 4 * kScrH + kScrPart;

}  // namespace

// The scratch itself (each device holds its own copy for the life of the process).
static __device__ __align__(256) unsigned char scratch[kStaticBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_static_mu;
void *g_static_ptr[kMaxDevices] = {};

// Device address of this device's copy of `scratch` (looked up on first use per device).
int static_scratch(void **out)
{
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(BBX_EDEVICE, "device %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_static_mu);
    if (!g_static_ptr[dev]) {
        void *p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress");
        if (!p) return fail(BBX_EDEVICE, "no device address for the static scratch");
        g_static_ptr[dev] = p;
    }
    *out = g_static_ptr[dev];
    return BBX_OK;
}

}  // namespace

extern "C" {

int bbx_mlp_grad_static(bbx_mlp *m, const float *X_dev, const float *T_dev, int64_t n,
                        float *grad_dev, double *loss_dev)
{
    try {
        g_err.clear();
        if (!m || !X_dev || !T_dev) return fail(BBX_EINVAL, "NULL argument");
        if (n < 1 || n > kStaticBatch)
            return fail(BBX_EINVAL, "n must be in [1, %lld] (the static scratch holds %lld samples)",
                        (long long)kStaticBatch, (long long)kStaticBatch);
        void *base = nullptr;
        int rc = static_scratch(&base);
        if (rc) return rc;
        unsigned char *p = (unsigned char *)base;
        MlpScratch w;
        w.xb = (__bf16 *)p;   p += kScrXb;
        w.tt = (float *)p;    p += kScrTt;
        w.xf = (__bf16 *)p;   p += kScrXf;
        w.dO = (__bf16 *)p;   p += kScrDo;
        w.h1 = (__bf16 *)p;   p += kScrH;
        w.h2 = (__bf16 *)p;   p += kScrH;
        w.dz1 = (__bf16 *)p;  p += kScrH;
        w.dz2 = (__bf16 *)p;  p += kScrH;
        w.part = (float *)p;
        // every scratch element the kernels read is written earlier in the same call
        // (padding samples included), so nothing needs clearing first
        HIP_TRY(mlp_grad(m->dev, w, 0, X_dev, T_dev, n, n, 0, 0, m->d_g, m->d_loss, m->stream),
                "gradient");
        if (grad_dev)
            HIP_TRY(hipMemcpyAsync(grad_dev, m->d_g, m->np * sizeof(float), hipMemcpyDeviceToDevice,
                                   m->stream), "hipMemcpyAsync");
        if (loss_dev)
            HIP_TRY(hipMemcpyAsync(loss_dev, m->d_loss, sizeof(double), hipMemcpyDeviceToDevice,
                                   m->stream), "hipMemcpyAsync");
        return BBX_OK;
    } catch (...) {
        return fail(BBX_EDEVICE, "unexpected failure");
    }
}

}  // extern "C"
