// Host side of the batched 2D ensemble: validation, layout, tile tables, graph
// capture and replay, autotuning and readout.  Every entry point catches
// everything: no C++ exception crosses the C ABI.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "../../include/bbx.h"
#include "ens_internal.h"

using namespace bbx;

namespace {

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    return api_error(code, buf);
}

int hip_fail(hipError_t e, const char *what)
{
    return fail(e == hipErrorOutOfMemory ? BBX_ENOMEM : BBX_EDEVICE, "%s: %s", what,
                hipGetErrorString(e));
}

#define HIP_TRY(expr, what)                              \
    do {                                                 \
        hipError_t e_ = (expr);                          \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

int ens_nvar(int m)
{
    switch (m) {
    case BBX_MODEL_NONE: return 1;
    case BBX_MODEL_BARKLEY: return 2;
    case BBX_MODEL_ZFK: return 1;
    case BBX_MODEL_FHN: return 2;
    case BBX_MODEL_FK4: return 4;
    default: return -1;
    }
}

int ens_nparams(int m)
{
    switch (m) {
    case BBX_MODEL_NONE: return 0;
    case BBX_MODEL_BARKLEY: return 3;
    case BBX_MODEL_ZFK: return 1;
    case BBX_MODEL_FHN: return 3;
    case BBX_MODEL_FK4: return 4;
    default: return -1;
    }
}

int64_t steps_of(double t, double dt) { return (int64_t)llround(t / dt); }

struct HostStim {
    int x0, x1, y0, y1;
    double amp;
    int64_t n0, len, per, count;
};

// max over the neighbourhood classes of a voxel (each of the four face
// neighbours present or not) of sum_q |W_q| including the centre weight, for
// the 9-point weights of a uniform 2D tensor.
double gershgorin_2d(double cxx, double cyy, double cxy)
{
    double best = 0;
    for (int m = 0; m < 16; m++) {
        const bool px = m & 1, mx = m & 2, py = m & 4, my = m & 8;
        double off = 0, c = 0;
        auto add = [&](bool on, double w) {
            if (!on) return;
            off += fabs(w);
            c -= w;
        };
        add(px, cxx);
        add(mx, cxx);
        add(py, cyy);
        add(my, cyy);
        add(px && py, cxy);
        add(mx && my, cxy);
        add(px && my, -cxy);
        add(mx && py, -cxy);
        best = std::max(best, off + fabs(c));
    }
    return best;
}

}  // namespace

struct bbx_ensemble {
    int ntis = 0, prec = 0, es = 4, model = 0, nvar = 1;
    double h = 0, dt = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::vector<int> nx, ny;
    std::vector<int64_t> off;
    std::vector<double> cxx, cyy, cxy, prm;
    std::vector<std::vector<HostStim>> stims;
    int64_t nvox = 0, pitch = 0;

    void *d_V[2] = {nullptr, nullptr};
    void *d_st = nullptr;
    void *d_tis = nullptr, *d_stims = nullptr;
    int4 *d_tiles = nullptr;
    int64_t *d_nbase = nullptr;
    int *d_flag = nullptr;
    uint8_t *d_status = nullptr;
    void *d_at = nullptr, *d_vmax = nullptr, *d_apd = nullptr, *d_vrep = nullptr;

    int variant = BBX_ENS_TILE_64x4, ntile = 0, per_xcd = 0, tile_cap = 0;
    int rec = 0;
    double theta = NAN;
    int64_t n = 0;                   // steps taken (host mirror of *d_nbase)
    int chunk = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    bool graph_dirty = true;
    size_t bytes = 0;
};

namespace {

template <typename P>
hipError_t dalloc(bbx_ensemble *e, P **p, size_t bytes)
{
    void *q = nullptr;
    hipError_t r = hipMalloc(&q, bytes ? bytes : 1);
    if (r == hipSuccess) {
        *p = (P *)q;
        e->bytes += bytes;
    }
    return r;
}

void dfree(void *p)
{
    if (p) (void)hipFree(p);
}

void drop_graph(bbx_ensemble *e)
{
    if (e->gexec) (void)hipGraphExecDestroy(e->gexec);
    if (e->graph) (void)hipGraphDestroy(e->graph);
    e->gexec = nullptr;
    e->graph = nullptr;
    e->graph_dirty = true;
}

void release(bbx_ensemble *e)
{
    if (e->stream) (void)hipStreamSynchronize(e->stream);
    drop_graph(e);
    void *bufs[] = {e->d_V[0], e->d_V[1], e->d_st, e->d_tis, e->d_stims, e->d_tiles, e->d_nbase,
                    e->d_flag, e->d_status, e->d_at, e->d_vmax, e->d_apd, e->d_vrep};
    for (void *p : bufs) dfree(p);
    if (e->own_stream && e->stream) (void)hipStreamDestroy(e->stream);
    delete e;
}

// Tile table of a variant: tissue after tissue, tiles row by row.
std::vector<int4> make_tiles(const bbx_ensemble *e, int variant)
{
    int tx, ty;
    ens_tile_shape(variant, &tx, &ty);
    std::vector<int4> t;
    for (int i = 0; i < e->ntis; i++)
        for (int y0 = 0; y0 < e->ny[i]; y0 += ty)
            for (int x0 = 0; x0 < e->nx[i]; x0 += tx) t.push_back(make_int4(i, x0, y0, 0));
    return t;
}

int max_tiles(const bbx_ensemble *e)
{
    size_t m = 0;
    for (int v = 0; v < BBX_ENS_NVARIANT; v++) m = std::max(m, make_tiles(e, v).size());
    return (int)m;
}

// Upload the tile table of `variant` into buf (capacity e->tile_cap); returns the count.
int upload_tiles(bbx_ensemble *e, int variant, int4 *buf, int *ntile)
{
    std::vector<int4> t = make_tiles(e, variant);
    if ((int)t.size() > e->tile_cap) return fail(BBX_EINVAL, "tile table exceeds its capacity");
    HIP_TRY(hipMemcpyAsync(buf, t.data(), t.size() * sizeof(int4), hipMemcpyHostToDevice, e->stream),
            "hipMemcpyAsync");
    HIP_TRY(hipStreamSynchronize(e->stream), "hipStreamSynchronize");
    *ntile = (int)t.size();
    return BBX_OK;
}

template <typename T>
int upload_tables(bbx_ensemble *e)
{
    std::vector<EnsTissue<T>> tis(e->ntis);
    std::vector<EnsStim<T>> st;
    for (int i = 0; i < e->ntis; i++) {
        EnsTissue<T> &t = tis[i];
        t.off = e->off[i];
        t.nx = e->nx[i];
        t.ny = e->ny[i];
        t.cxx = (T)e->cxx[i];
        t.cyy = (T)e->cyy[i];
        t.cxy = (T)e->cxy[i];
        for (int k = 0; k < kEnsParams; k++) t.prm[k] = (T)e->prm[(size_t)i * kEnsParams + k];
        t.s0 = (int)st.size();
        for (const HostStim &h : e->stims[i])
            st.push_back({h.x0, h.x1, h.y0, h.y1, (T)h.amp, h.n0, h.len, h.per, h.count});
        t.s1 = (int)st.size();
    }
    HIP_TRY(hipMemcpyAsync(e->d_tis, tis.data(), tis.size() * sizeof(EnsTissue<T>),
                           hipMemcpyHostToDevice, e->stream), "hipMemcpyAsync");
    if (!st.empty())
        HIP_TRY(hipMemcpyAsync(e->d_stims, st.data(), st.size() * sizeof(EnsStim<T>),
                               hipMemcpyHostToDevice, e->stream), "hipMemcpyAsync");
    HIP_TRY(hipStreamSynchronize(e->stream), "hipStreamSynchronize");
    return BBX_OK;
}

int upload(bbx_ensemble *e) { return e->prec ? upload_tables<double>(e) : upload_tables<float>(e); }

template <typename T>
EnsArgs<T> make_args(const bbx_ensemble *e)
{
    EnsArgs<T> a = {};
    a.tiles = e->d_tiles;
    a.ntile = e->ntile;
    a.per_xcd = e->per_xcd;
    a.tis = (const EnsTissue<T> *)e->d_tis;
    a.stims = (const EnsStim<T> *)e->d_stims;
    a.V0 = (T *)e->d_V[0];
    a.V1 = (T *)e->d_V[1];
    a.st = (T *)e->d_st;
    a.pitch = e->pitch;
    a.dt = (T)e->dt;
    a.dt64 = e->dt;
    a.nbase = e->d_nbase;
    a.rec = e->rec;
    a.theta = (T)e->theta;
    a.status = e->d_status;
    a.at = (T *)e->d_at;
    a.vmax = (T *)e->d_vmax;
    a.apd = (T *)e->d_apd;
    a.vrep = (T *)e->d_vrep;
    // Measured on the 96-tissue FK4 ensemble (384 MB of state): 195 -> 182 us per step.
    a.nt = (double)e->nvox * e->nvar * sizeof(T) > kInfinityCacheBytes;
    return a;
}

// Launch k steps directly (j = 0..k-1 of a batch) and advance the device clock.
template <typename T>
int launch_batch(bbx_ensemble *e, const EnsArgs<T> &a, int variant, int64_t k, int64_t *nbase)
{
    if (k <= 0) return BBX_OK;
    for (int64_t j = 0; j < k; j++)
        HIP_TRY(launch_ens_step<T>(e->model, variant, a, (int)j, e->stream), "ensemble step launch");
    HIP_TRY(launch_ens_advance(nbase, k, e->stream), "ensemble clock launch");
    return BBX_OK;
}

template <typename T>
int capture(bbx_ensemble *e)
{
    drop_graph(e);
    const EnsArgs<T> a = make_args<T>(e);
    HIP_TRY(hipStreamBeginCapture(e->stream, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
    int rc = launch_batch<T>(e, a, e->variant, e->chunk, e->d_nbase);
    hipGraph_t g = nullptr;
    hipError_t r = hipStreamEndCapture(e->stream, &g);
    if (rc != BBX_OK) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (r != hipSuccess) return hip_fail(r, "hipStreamEndCapture");
    e->graph = g;
    r = hipGraphInstantiate(&e->gexec, g, nullptr, nullptr, 0);
    if (r != hipSuccess) {
        drop_graph(e);
        return hip_fail(r, "hipGraphInstantiate");
    }
    e->graph_dirty = false;
    return BBX_OK;
}

template <typename T>
int step_impl(bbx_ensemble *e, int64_t nsteps)
{
    int64_t left = nsteps;
    if (e->chunk > 0 && left >= e->chunk) {
        if (e->graph_dirty || !e->gexec) {
            int rc = capture<T>(e);
            if (rc) return rc;
        }
        while (left >= e->chunk) {
            HIP_TRY(hipGraphLaunch(e->gexec, e->stream), "hipGraphLaunch");
            left -= e->chunk;
        }
    }
    int rc = launch_batch<T>(e, make_args<T>(e), e->variant, left, e->d_nbase);
    if (rc) return rc;
    e->n += nsteps;
    return BBX_OK;
}

template <typename T>
int tune_impl(bbx_ensemble *e, int steps, int *best, double *times)
{
    // scratch copies of the state and clock; the recorder is off
    const size_t vb = (size_t)e->nvox * sizeof(T), sb = (size_t)(e->nvar - 1) * e->pitch * sizeof(T);
    void *sV0 = nullptr, *sV1 = nullptr, *sst = nullptr;
    int64_t *snb = nullptr;
    int4 *stl = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    int rc = BBX_OK;
    double t_ms[BBX_ENS_NVARIANT];
    auto cleanup = [&]() {
        (void)hipStreamSynchronize(e->stream);
        dfree(sV0);
        dfree(sV1);
        dfree(sst);
        dfree(snb);
        dfree(stl);
        if (ev0) (void)hipEventDestroy(ev0);
        if (ev1) (void)hipEventDestroy(ev1);
    };
    hipError_t r = hipMalloc(&sV0, vb);
    if (r == hipSuccess) r = hipMalloc(&sV1, vb);
    if (r == hipSuccess) r = hipMalloc(&sst, sb ? sb : 1);
    if (r == hipSuccess) r = hipMalloc((void **)&snb, sizeof(int64_t));
    if (r == hipSuccess) r = hipMalloc((void **)&stl, (size_t)e->tile_cap * sizeof(int4));
    if (r == hipSuccess) r = hipEventCreate(&ev0);
    if (r == hipSuccess) r = hipEventCreate(&ev1);
    if (r == hipSuccess) r = hipMemcpyAsync(sV0, e->d_V[0], vb, hipMemcpyDeviceToDevice, e->stream);
    if (r == hipSuccess) r = hipMemcpyAsync(sV1, e->d_V[1], vb, hipMemcpyDeviceToDevice, e->stream);
    if (r == hipSuccess && sb) r = hipMemcpyAsync(sst, e->d_st, sb, hipMemcpyDeviceToDevice, e->stream);
    if (r == hipSuccess) r = hipMemcpyAsync(snb, e->d_nbase, sizeof(int64_t), hipMemcpyDeviceToDevice, e->stream);
    if (r != hipSuccess) {
        rc = hip_fail(r, "autotune set-up");
        cleanup();
        return rc;
    }
    EnsArgs<T> a = make_args<T>(e);
    a.V0 = (T *)sV0;
    a.V1 = (T *)sV1;
    a.st = (T *)sst;
    a.nbase = snb;
    a.rec = 0;
    a.tiles = stl;
    int pick = 0;
    for (int v = 0; v < BBX_ENS_NVARIANT && rc == BBX_OK; v++) {
        int nt = 0;
        rc = upload_tiles(e, v, stl, &nt);
        if (rc) break;
        a.ntile = nt;
        a.per_xcd = (nt + kXcd - 1) / kXcd;
        rc = launch_batch<T>(e, a, v, 2, snb);          // warm-up
        if (rc) break;
        r = hipEventRecord(ev0, e->stream);
        if (r == hipSuccess) rc = launch_batch<T>(e, a, v, steps, snb);
        if (rc) break;
        if (r == hipSuccess) r = hipEventRecord(ev1, e->stream);
        if (r == hipSuccess) r = hipEventSynchronize(ev1);
        float ms = 0;
        if (r == hipSuccess) r = hipEventElapsedTime(&ms, ev0, ev1);
        if (r != hipSuccess) {
            rc = hip_fail(r, "autotune timing");
            break;
        }
        t_ms[v] = ms;
        if (ms < t_ms[pick]) pick = v;
    }
    cleanup();
    if (rc) return rc;
    if (times)
        for (int v = 0; v < BBX_ENS_NVARIANT; v++) times[v] = t_ms[v];
    if (best) *best = pick;
    return bbx_ensemble_variant_set(e, pick);
}

template <typename T>
int readout_impl(bbx_ensemble *e, int what, int tissue, int var, void *out, size_t count)
{
    const int64_t np = (int64_t)e->nx[tissue] * e->ny[tissue], o = e->off[tissue];
    if (what == BBX_READ_STATUS) {
        if ((int64_t)count < np) return fail(BBX_EINVAL, "out holds %zu elements, need %lld", count, (long long)np);
        HIP_TRY(hipMemcpyAsync(out, e->d_status + o, np, hipMemcpyDeviceToHost, e->stream), "hipMemcpyAsync");
        HIP_TRY(hipStreamSynchronize(e->stream), "hipStreamSynchronize");
        return BBX_OK;
    }
    const T *src = nullptr;
    switch (what) {
    case BBX_READ_VAR:
        src = var == 0 ? (const T *)e->d_V[e->n & 1] + o : (const T *)e->d_st + (var - 1) * e->pitch + o;
        break;
    case BBX_READ_ACT_TIME: src = (const T *)e->d_at + o; break;
    case BBX_READ_APD90: src = (const T *)e->d_apd + o; break;
    case BBX_READ_VMAX: src = (const T *)e->d_vmax + o; break;
    }
    if ((int64_t)count < np) return fail(BBX_EINVAL, "out holds %zu elements, need %lld", count, (long long)np);
    std::vector<T> tmp(np);
    HIP_TRY(hipMemcpyAsync(tmp.data(), src, np * sizeof(T), hipMemcpyDeviceToHost, e->stream), "hipMemcpyAsync");
    HIP_TRY(hipStreamSynchronize(e->stream), "hipStreamSynchronize");
    double *d = (double *)out;
    for (int64_t i = 0; i < np; i++) d[i] = (double)tmp[i];
    return BBX_OK;
}

template <typename T>
int recording_impl(bbx_ensemble *e, double theta)
{
    const size_t nb = (size_t)e->nvox;
    hipError_t r = hipSuccess;
    if (!e->d_status) {
        r = dalloc(e, &e->d_status, nb);
        if (r == hipSuccess) r = dalloc(e, &e->d_at, nb * sizeof(T));
        if (r == hipSuccess) r = dalloc(e, &e->d_vmax, nb * sizeof(T));
        if (r == hipSuccess) r = dalloc(e, &e->d_apd, nb * sizeof(T));
        if (r == hipSuccess) r = dalloc(e, &e->d_vrep, nb * sizeof(T));
        if (r != hipSuccess) return hip_fail(r, "hipMalloc");
    }
    HIP_TRY(hipMemsetAsync(e->d_status, 0, nb, e->stream), "hipMemsetAsync");
    HIP_TRY(launch_fill<T>((T *)e->d_at, (T)NAN, (int64_t)nb, e->stream), "fill");
    HIP_TRY(launch_fill<T>((T *)e->d_vmax, (T)NAN, (int64_t)nb, e->stream), "fill");
    HIP_TRY(launch_fill<T>((T *)e->d_apd, (T)NAN, (int64_t)nb, e->stream), "fill");
    HIP_TRY(hipMemcpyAsync(e->d_vrep, e->d_V[e->n & 1], nb * sizeof(T), hipMemcpyDeviceToDevice, e->stream),
            "hipMemcpyAsync");
    e->rec = 1;
    e->theta = theta;
    e->graph_dirty = true;
    return BBX_OK;
}

}  // namespace

extern "C" {

int bbx_ensemble_create(int ntissue, const int *nx, const int *ny, double h, const double *Dpar,
                        const double *Dperp, const double *angle, int model, const double *params,
                        int nparams, double dt, int precision, void *hip_stream, bbx_ensemble **out)
{
    try {
        api_clear_error();
        if (!out) return fail(BBX_EINVAL, "out is NULL");
        *out = nullptr;
        if (ntissue < 1) return fail(BBX_EINVAL, "ntissue must be >= 1");
        if (!nx || !ny || !Dpar || !Dperp || !angle) return fail(BBX_EINVAL, "a per-tissue array is NULL");
        if (!(h > 0) || !isfinite(h)) return fail(BBX_EINVAL, "h must be positive");
        if (!(dt > 0) || !isfinite(dt)) return fail(BBX_EINVAL, "dt must be positive");
        if (precision != BBX_FP32 && precision != BBX_FP64) return fail(BBX_EINVAL, "bad precision");
        if (model == BBX_MODEL_CRN) return fail(BBX_ENOTSUP, "the ensemble runs the 2D models (not CRN)");
        const int nv = ens_nvar(model), np = ens_nparams(model);
        if (nv < 0) return fail(BBX_EINVAL, "unknown model %d", model);
        if (nparams != np) return fail(BBX_EINVAL, "model %d takes %d parameters, got %d", model, np, nparams);
        if (np > 0 && !params) return fail(BBX_EINVAL, "params is NULL");
        int64_t total = 0;
        for (int i = 0; i < ntissue; i++) {
            if (nx[i] < 1 || ny[i] < 1) return fail(BBX_EINVAL, "tissue %d has size %d x %d", i, nx[i], ny[i]);
            if (!(Dpar[i] >= 0) || !(Dperp[i] >= 0) || !isfinite(Dpar[i]) || !isfinite(Dperp[i]) ||
                !isfinite(angle[i]))
                return fail(BBX_EINVAL, "tissue %d: diffusion coefficients and angle must be finite, D >= 0", i);
            for (int k = 0; k < np; k++)
                if (!isfinite(params[(size_t)i * np + k])) return fail(BBX_EINVAL, "tissue %d: parameter %d not finite", i, k);
            total += (int64_t)nx[i] * ny[i];
        }
        if (total >= (int64_t)1 << 31) return fail(BBX_EINVAL, "more than 2^31 voxels in total");

        bbx_ensemble *e = new bbx_ensemble();
        e->ntis = ntissue;
        e->prec = precision;
        e->es = precision ? 8 : 4;
        e->model = model;
        e->nvar = nv;
        e->h = h;
        e->dt = dt;
        e->nx.assign(nx, nx + ntissue);
        e->ny.assign(ny, ny + ntissue);
        e->off.resize(ntissue);
        e->cxx.resize(ntissue);
        e->cyy.resize(ntissue);
        e->cxy.resize(ntissue);
        e->prm.assign((size_t)ntissue * kEnsParams, 0.0);
        e->stims.resize(ntissue);
        double wmax = 0;
        for (int i = 0; i < ntissue; i++) {
            e->off[i] = e->nvox;
            e->nvox += (int64_t)nx[i] * ny[i];
            const double c = cos(angle[i]), s = sin(angle[i]), dd = Dpar[i] - Dperp[i], ih2 = 1.0 / (h * h);
            e->cxx[i] = (Dperp[i] + dd * c * c) * ih2;
            e->cyy[i] = (Dperp[i] + dd * s * s) * ih2;
            e->cxy[i] = dd * c * s * ih2 * 0.5;
            for (int k = 0; k < np; k++) e->prm[(size_t)i * kEnsParams + k] = params[(size_t)i * np + k];
            wmax = std::max(wmax, gershgorin_2d(e->cxx[i], e->cyy[i], e->cxy[i]));
        }
        if (wmax > 0 && dt > 2.0 / wmax) {
            delete e;
            return fail(BBX_EUNSTABLE, "dt %g exceeds the explicit diffusion bound %g", dt, 2.0 / wmax);
        }
        e->pitch = (e->nvox + 63) / 64 * 64;

        int rc = BBX_OK;
        hipError_t r = hipSuccess;
        if (hip_stream) {
            e->stream = (hipStream_t)hip_stream;
        } else {
            r = hipStreamCreate(&e->stream);
            if (r != hipSuccess) {
                delete e;
                return hip_fail(r, "hipStreamCreate");
            }
            e->own_stream = true;
        }
        const size_t es = e->es;
        e->tile_cap = max_tiles(e);
        if (r == hipSuccess) r = dalloc(e, &e->d_V[0], e->nvox * es);
        if (r == hipSuccess) r = dalloc(e, &e->d_V[1], e->nvox * es);
        if (r == hipSuccess) r = dalloc(e, &e->d_st, (size_t)(nv - 1) * e->pitch * es);
        if (r == hipSuccess)
            r = dalloc(e, &e->d_tis, ntissue * (precision ? sizeof(EnsTissue<double>) : sizeof(EnsTissue<float>)));
        if (r == hipSuccess)
            r = dalloc(e, &e->d_stims, (size_t)ntissue * kEnsMaxStim *
                                           (precision ? sizeof(EnsStim<double>) : sizeof(EnsStim<float>)));
        if (r == hipSuccess) r = dalloc(e, &e->d_tiles, (size_t)e->tile_cap * sizeof(int4));
        if (r == hipSuccess) r = dalloc(e, &e->d_nbase, sizeof(int64_t));
        if (r == hipSuccess) r = dalloc(e, &e->d_flag, sizeof(int));
        if (r == hipSuccess) r = hipMemsetAsync(e->d_V[0], 0, e->nvox * es, e->stream);
        if (r == hipSuccess) r = hipMemsetAsync(e->d_V[1], 0, e->nvox * es, e->stream);
        if (r == hipSuccess && nv > 1) r = hipMemsetAsync(e->d_st, 0, (size_t)(nv - 1) * e->pitch * es, e->stream);
        if (r == hipSuccess) r = hipMemsetAsync(e->d_nbase, 0, sizeof(int64_t), e->stream);
        if (r != hipSuccess) {
            rc = hip_fail(r, "ensemble allocation");
            release(e);
            return rc;
        }
        rc = upload(e);
        if (rc == BBX_OK) rc = upload_tiles(e, e->variant, e->d_tiles, &e->ntile);
        if (rc != BBX_OK) {
            release(e);
            return rc;
        }
        e->per_xcd = (e->ntile + kXcd - 1) / kXcd;
        *out = e;
        return BBX_OK;
    } catch (...) {
        return fail(BBX_ENOMEM, "host allocation failed");
    }
}

int bbx_ensemble_state_set(bbx_ensemble *e, int tissue, int var, const double *values)
{
    try {
        api_clear_error();
        if (!e) return fail(BBX_EINVAL, "ensemble is NULL");
        if (!values) return fail(BBX_EINVAL, "values is NULL");
        if (tissue < 0 || tissue >= e->ntis) return fail(BBX_EINVAL, "tissue %d out of range", tissue);
        if (var < 0 || var >= e->nvar) return fail(BBX_EINVAL, "var %d out of range (nvar %d)", var, e->nvar);
        const int64_t np = (int64_t)e->nx[tissue] * e->ny[tissue], o = e->off[tissue];
        for (int64_t i = 0; i < np; i++)
            if (!isfinite(values[i])) return fail(BBX_EINVAL, "value %lld is not finite", (long long)i);
        const size_t es = e->es;
        char *dst = (char *)(var == 0 ? e->d_V[e->n & 1] : (char *)e->d_st + (size_t)(var - 1) * e->pitch * es);
        dst += (size_t)o * es;
        if (e->prec) {
            HIP_TRY(hipMemcpyAsync(dst, values, np * es, hipMemcpyHostToDevice, e->stream), "hipMemcpyAsync");
            HIP_TRY(hipStreamSynchronize(e->stream), "hipStreamSynchronize");
        } else {
            std::vector<float> tmp(values, values + np);
            HIP_TRY(hipMemcpyAsync(dst, tmp.data(), np * es, hipMemcpyHostToDevice, e->stream), "hipMemcpyAsync");
            HIP_TRY(hipStreamSynchronize(e->stream), "hipStreamSynchronize");
        }
        return BBX_OK;
    } catch (...) {
        return fail(BBX_ENOMEM, "host allocation failed");
    }
}

int bbx_ensemble_stimulus_add(bbx_ensemble *e, int tissue, int x0, int x1, int y0, int y1,
                              double amplitude, double t_start, double duration, double period, int count)
{
    try {
        api_clear_error();
        if (!e) return fail(BBX_EINVAL, "ensemble is NULL");
        if (tissue < 0 || tissue >= e->ntis) return fail(BBX_EINVAL, "tissue %d out of range", tissue);
        if ((int)e->stims[tissue].size() >= kEnsMaxStim)
            return fail(BBX_EINVAL, "at most %d stimuli per tissue", kEnsMaxStim);
        if (!(x0 >= 0 && x0 < x1 && x1 <= e->nx[tissue] && y0 >= 0 && y0 < y1 && y1 <= e->ny[tissue]))
            return fail(BBX_EINVAL, "stimulus rectangle outside tissue %d", tissue);
        if (!isfinite(amplitude) || !isfinite(t_start) || !isfinite(duration) || !isfinite(period))
            return fail(BBX_EINVAL, "stimulus values must be finite");
        if (t_start < 0 || duration < 0 || period < 0 || count < 0)
            return fail(BBX_EINVAL, "stimulus times and count must be >= 0");
        HostStim s = {x0, x1, y0, y1, amplitude, steps_of(t_start, e->dt), steps_of(duration, e->dt),
                      period > 0 ? steps_of(period, e->dt) : 0, count};
        e->stims[tissue].push_back(s);
        int rc = upload(e);
        if (rc) {
            e->stims[tissue].pop_back();
            return rc;
        }
        e->graph_dirty = true;
        return BBX_OK;
    } catch (...) {
        return fail(BBX_ENOMEM, "host allocation failed");
    }
}

int bbx_ensemble_recording_set(bbx_ensemble *e, double theta)
{
    try {
        api_clear_error();
        if (!e) return fail(BBX_EINVAL, "ensemble is NULL");
        if (!isfinite(theta)) return fail(BBX_EINVAL, "theta must be finite");
        return e->prec ? recording_impl<double>(e, theta) : recording_impl<float>(e, theta);
    } catch (...) {
        return fail(BBX_ENOMEM, "host allocation failed");
    }
}

int bbx_ensemble_graph_set(bbx_ensemble *e, int chunk)
{
    api_clear_error();
    if (!e) return fail(BBX_EINVAL, "ensemble is NULL");
    if (chunk < 0 || chunk > 4096 || (chunk & 1)) return fail(BBX_EINVAL, "chunk must be even, 0..4096");
    if (chunk != e->chunk) drop_graph(e);
    e->chunk = chunk;
    return BBX_OK;
}

int bbx_ensemble_variant_set(bbx_ensemble *e, int variant)
{
    try {
        api_clear_error();
        if (!e) return fail(BBX_EINVAL, "ensemble is NULL");
        if (variant < 0 || variant >= BBX_ENS_NVARIANT) return fail(BBX_EINVAL, "unknown variant %d", variant);
        HIP_TRY(hipStreamSynchronize(e->stream), "hipStreamSynchronize");
        int nt = 0;
        int rc = upload_tiles(e, variant, e->d_tiles, &nt);
        if (rc) return rc;
        e->variant = variant;
        e->ntile = nt;
        e->per_xcd = (nt + kXcd - 1) / kXcd;
        e->graph_dirty = true;
        return BBX_OK;
    } catch (...) {
        return fail(BBX_ENOMEM, "host allocation failed");
    }
}

int bbx_ensemble_tune(bbx_ensemble *e, int steps, int *variant, double *times_ms)
{
    try {
        api_clear_error();
        if (!e) return fail(BBX_EINVAL, "ensemble is NULL");
        if (steps < 1 || steps > 100000) return fail(BBX_EINVAL, "steps must be in 1..100000");
        return e->prec ? tune_impl<double>(e, steps, variant, times_ms)
                       : tune_impl<float>(e, steps, variant, times_ms);
    } catch (...) {
        return fail(BBX_ENOMEM, "host allocation failed");
    }
}

int bbx_ensemble_step(bbx_ensemble *e, int64_t nsteps)
{
    try {
        api_clear_error();
        if (!e) return fail(BBX_EINVAL, "ensemble is NULL");
        if (nsteps < 0) return fail(BBX_EINVAL, "nsteps must be >= 0");
        if (nsteps == 0) return BBX_OK;
        return e->prec ? step_impl<double>(e, nsteps) : step_impl<float>(e, nsteps);
    } catch (...) {
        return fail(BBX_ENOMEM, "host allocation failed");
    }
}

int bbx_ensemble_readout(bbx_ensemble *e, int what, int tissue, int var, void *out, size_t count)
{
    try {
        api_clear_error();
        if (!e) return fail(BBX_EINVAL, "ensemble is NULL");
        if (!out) return fail(BBX_EINVAL, "out is NULL");
        switch (what) {
        case BBX_READ_STEP:
            if (count < 1) return fail(BBX_EINVAL, "out holds no element");
            *(int64_t *)out = e->n;
            return BBX_OK;
        case BBX_READ_NAN_FLAG: {
            if (count < 1) return fail(BBX_EINVAL, "out holds no element");
            HIP_TRY(hipMemsetAsync(e->d_flag, 0, sizeof(int), e->stream), "hipMemsetAsync");
            if (e->prec)
                HIP_TRY(launch_nonfinite<double>((const double *)e->d_V[e->n & 1], nullptr, 1,
                                                 (const double *)e->d_st, e->nvar - 1, e->nvox, e->pitch,
                                                 e->d_flag, e->stream), "finite check");
            else
                HIP_TRY(launch_nonfinite<float>((const float *)e->d_V[e->n & 1], nullptr, 1,
                                                (const float *)e->d_st, e->nvar - 1, e->nvox, e->pitch,
                                                e->d_flag, e->stream), "finite check");
            HIP_TRY(hipMemcpyAsync(out, e->d_flag, sizeof(int), hipMemcpyDeviceToHost, e->stream), "hipMemcpyAsync");
            HIP_TRY(hipStreamSynchronize(e->stream), "hipStreamSynchronize");
            return BBX_OK;
        }
        case BBX_READ_VAR:
        case BBX_READ_ACT_TIME:
        case BBX_READ_APD90:
        case BBX_READ_VMAX:
        case BBX_READ_STATUS:
            break;
        default:
            return fail(BBX_EINVAL, "readout %d is not provided for ensembles", what);
        }
        if (tissue < 0 || tissue >= e->ntis) return fail(BBX_EINVAL, "tissue %d out of range", tissue);
        if (what == BBX_READ_VAR && (var < 0 || var >= e->nvar))
            return fail(BBX_EINVAL, "var %d out of range (nvar %d)", var, e->nvar);
        if (what != BBX_READ_VAR && !e->rec) return fail(BBX_ESTATE, "recording is off");
        return e->prec ? readout_impl<double>(e, what, tissue, var, out, count)
                       : readout_impl<float>(e, what, tissue, var, out, count);
    } catch (...) {
        return fail(BBX_ENOMEM, "host allocation failed");
    }
}

int bbx_ensemble_info(const bbx_ensemble *e, int what, int64_t *out)
{
    api_clear_error();
    if (!e || !out) return fail(BBX_EINVAL, "NULL argument");
    switch (what) {
    case BBX_ENS_INFO_VOXELS: *out = e->nvox; return BBX_OK;
    case BBX_ENS_INFO_TILES: *out = e->ntile; return BBX_OK;
    case BBX_ENS_INFO_VARIANT: *out = e->variant; return BBX_OK;
    case BBX_ENS_INFO_DEVICE_BYTES: *out = (int64_t)e->bytes; return BBX_OK;
    case BBX_ENS_INFO_GRAPH_CHUNK: *out = e->chunk; return BBX_OK;
    case BBX_ENS_INFO_NVAR: *out = e->nvar; return BBX_OK;
    default: return fail(BBX_EINVAL, "unknown info %d", what);
    }
}

void bbx_ensemble_destroy(bbx_ensemble *e)
{
    if (e) release(e);
}

}  // extern "C"
