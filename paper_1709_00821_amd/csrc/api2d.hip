// Host side of the 2D library: descriptor validation, workspace layout, the
// compact plasma support, time loop (eager or replayed from a captured HIP
// graph), probe DFT windows, field read-back.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "../../include/fdtd_plasma2d.h"
#include "internal.h"
#include "internal2d.h"

using namespace fdtdp;

namespace {

thread_local std::string g_err2;

int fail2(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err2 = buf;
    return code;
}

#define HIP_TRY2(expr)                                                                   \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess)                                                            \
            return fail2(FDTD_E_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));  \
    } while (0)

constexpr int64_t kAlign2 = 256;
constexpr int kSB2 = 2048;     // probe samples per DFT window

int64_t rup(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

struct Lay {
    int64_t total = 0;
    int64_t take(int64_t b)
    {
        const int64_t o = total;
        total += rup(std::max<int64_t>(b, 16), kAlign2);
        return o;
    }
};

struct Plan2 {
    Lay L;
    int ncomp = 1, nh = 2, es = 8;
    int64_t N = 0, S = 0;
    std::vector<int2> span;
    std::vector<int64_t> rowoff;
    int64_t o_E[2] = {0, 0}, o_H[2] = {0, 0}, o_span = 0, o_rowoff = 0, o_wp2[2] = {0, 0}, o_nu[2] = {0, 0},
            o_J[2] = {0, 0}, o_probes = 0, o_freqs = 0, o_samp = 0, o_X = 0, o_Xtmp = 0, o_tw = 0;
};

int validate2(const fdtd2d_desc *d)
{
    if (!d) return fail2(FDTD_E_INVALID, "descriptor is NULL");
    if (d->struct_size != sizeof(fdtd2d_desc))
        return fail2(FDTD_E_INVALID, "struct_size %u != %zu (header/library mismatch)", d->struct_size,
                     sizeof(fdtd2d_desc));
    if (d->mode != FDTD2D_TM && d->mode != FDTD2D_TE) return fail2(FDTD_E_INVALID, "mode %d", d->mode);
    if (d->precision != FDTD_F64 && d->precision != FDTD_F32)
        return fail2(FDTD_E_INVALID, "precision %d (FDTD_F64 or FDTD_F32)", d->precision);
    if (d->nx < 2 || d->ny < 2 || d->nx > (1 << 20) || d->ny > (1 << 20) || d->nx * d->ny > ((int64_t)1 << 32))
        return fail2(FDTD_E_INVALID, "grid %lld x %lld out of range", (long long)d->nx, (long long)d->ny);
    if (!(d->d > 0.0) || !(d->dt > 0.0) || !std::isfinite(d->d) || !std::isfinite(d->dt))
        return fail2(FDTD_E_INVALID, "d and dt must be positive and finite");
    if (kC0 * d->dt / d->d > 1.0 / std::sqrt(2.0))
        return fail2(FDTD_E_UNSTABLE, "Courant number c dt/d = %.6g exceeds 1/sqrt(2)", kC0 * d->dt / d->d);
    if (!d->wp2 || !d->nu || (d->n_probes > 0 && !d->probes) || !d->freqs_hz)
        return fail2(FDTD_E_INVALID, "a host array pointer is NULL");
    if (d->n_probes < 0 || d->n_probes > 4096 || d->n_freqs < 1)
        return fail2(FDTD_E_INVALID, "need 0 <= n_probes <= 4096 and n_freqs >= 1");
    const int nc = d->mode == FDTD2D_TM ? 1 : 2;
    const int64_t N = d->nx * d->ny;
    for (int64_t k = 0; k < nc * N; ++k)
        if (!(d->wp2[k] >= 0.0) || !std::isfinite(d->wp2[k]) || !(d->nu[k] >= 0.0) || !std::isfinite(d->nu[k]))
            return fail2(FDTD_E_INVALID, "wp2 and nu must be finite and >= 0 (entry %lld)", (long long)k);
    if (d->has_src && (d->src_i < 0 || d->src_i >= d->nx || d->src_j < 0 || d->src_j >= d->ny))
        return fail2(FDTD_E_INVALID, "source (%lld, %lld) outside the grid", (long long)d->src_i,
                     (long long)d->src_j);
    if (d->has_src && !(std::isfinite(d->src_tau) && d->src_tau > 0 && std::isfinite(d->src_t0) &&
                        std::isfinite(d->src_amp)))
        return fail2(FDTD_E_INVALID, "source parameters must be finite with tau > 0");
    for (int p = 0; p < d->n_probes; ++p) {
        const int64_t *q = d->probes + 3 * p;
        if (q[0] < 0 || q[0] >= nc || q[1] < 0 || q[1] >= d->nx || q[2] < 0 || q[2] >= d->ny)
            return fail2(FDTD_E_INVALID, "probe %d (%lld, %lld, %lld) outside the grid or the mode", p,
                         (long long)q[0], (long long)q[1], (long long)q[2]);
    }
    for (int f = 0; f < d->n_freqs; ++f)
        if (!std::isfinite(d->freqs_hz[f])) return fail2(FDTD_E_INVALID, "freqs_hz[%d] not finite", f);
    return FDTD_OK;
}

int plan2(const fdtd2d_desc *d, Plan2 &p)
{
    int rc = validate2(d);
    if (rc) return rc;
    p.ncomp = d->mode == FDTD2D_TM ? 1 : 2;
    p.nh = d->mode == FDTD2D_TM ? 2 : 1;
    p.es = d->precision == FDTD_F64 ? 8 : 4;
    p.N = d->nx * d->ny;
    // compact plasma support: per row the span of cells where any component has wp2 > 0
    p.span.assign(d->nx, make_int2(0, 0));
    p.rowoff.assign(d->nx, 0);
    int64_t S = 0;
    for (int64_t i = 0; i < d->nx; ++i) {
        int64_t j0 = d->ny, j1 = 0;
        for (int c = 0; c < p.ncomp; ++c)
            for (int64_t j = 0; j < d->ny; ++j)
                if (d->wp2[c * p.N + i * d->ny + j] > 0.0) {
                    j0 = std::min(j0, j);
                    j1 = std::max(j1, j + 1);
                }
        if (j1 > j0) {
            p.span[i] = make_int2((int)j0, (int)j1);
            p.rowoff[i] = S;
            S += j1 - j0;
        }
    }
    p.S = S;
    Lay &L = p.L;
    L = Lay();
    for (int c = 0; c < p.ncomp; ++c) p.o_E[c] = L.take(p.es * p.N);
    for (int c = 0; c < p.nh; ++c) p.o_H[c] = L.take(p.es * p.N);
    p.o_span = L.take(8 * d->nx);
    p.o_rowoff = L.take(8 * d->nx);
    for (int c = 0; c < p.ncomp; ++c) {
        p.o_wp2[c] = L.take(8 * S);
        p.o_nu[c] = L.take(8 * S);
        p.o_J[c] = L.take(8 * S);
    }
    const int P = std::max(d->n_probes, 1);
    p.o_probes = L.take(24 * P);
    p.o_freqs = L.take(8 * d->n_freqs);
    p.o_samp = L.take(8 * (int64_t)P * kSB2);
    p.o_X = L.take(16 * (int64_t)P * d->n_freqs);
    p.o_Xtmp = L.take(16 * (int64_t)P * d->n_freqs);
    p.o_tw = L.take(16 * (int64_t)std::min(kSB2, kTwiddleChunk) * d->n_freqs);
    return FDTD_OK;
}

}  // namespace

struct fdtd2d {
    fdtd2d_desc d;
    hipStream_t stream = nullptr;
    bool owns = false;
    char *ws = nullptr;
    Plan2 p;
    Grid2 g;
    void *E[2] = {nullptr, nullptr}, *H[2] = {nullptr, nullptr};
    double *freqs = nullptr, *samp = nullptr;
    double2 *X = nullptr, *Xtmp = nullptr, *tw = nullptr;
    int64_t steps = 0, win_base = 0;
    bool tmp_valid = false;
    std::map<int64_t, hipGraphExec_t> graphs;
};

namespace {

Grids dft_view(const fdtd2d *h)
{
    Grids g{};
    g.samp = h->samp;
    g.SB = kSB2;
    g.dt = h->d.dt;
    return g;
}

void reset2(fdtd2d *h)
{
    for (int c = 0; c < h->p.ncomp; ++c) {
        launch_fill(h->E[c], rup(h->p.es * h->p.N, 16), h->stream);
        if (h->p.S) launch_fill(h->g.J[c], rup(8 * h->p.S, 16), h->stream);
    }
    for (int c = 0; c < h->p.nh; ++c) launch_fill(h->H[c], rup(h->p.es * h->p.N, 16), h->stream);
    const int P = std::max(h->d.n_probes, 1);
    launch_fill(h->X, rup(16 * (int64_t)P * h->d.n_freqs, 16), h->stream);
    h->steps = 0;
    h->win_base = 0;
}

void fold(fdtd2d *h, double2 *dst)
{
    const int count = (int)(h->steps - h->win_base);
    if (h->d.n_probes > 0 && count > 0)
        launch_dft(dft_view(h), h->freqs, h->d.n_freqs, h->win_base + 1, count, h->tw, dst, h->d.n_probes,
                   h->stream);
}

void to_tmp(fdtd2d *h)
{
    const int P = std::max(h->d.n_probes, 1);
    launch_copy(h->Xtmp, h->X, 16 * (int64_t)P * h->d.n_freqs, h->stream);
    fold(h, h->Xtmp);
}

template <typename T>
void advance2_t(fdtd2d *h, int64_t n)
{
    Fields2<T> f;
    for (int c = 0; c < 2; ++c) {
        f.E[c] = (T *)h->E[c];
        f.H[c] = (T *)h->H[c];
    }
    for (int64_t s = 0; s < n; ++s) {
        const int slot = (int)(h->steps - h->win_base);
        launch_step2d<T>(h->g, f, h->steps + 1, slot, h->stream);
        h->steps += 1;
        if (h->steps - h->win_base == kSB2) {
            fold(h, h->X);
            h->win_base = h->steps;
        }
    }
}

int advance2(fdtd2d *h, int64_t n)
{
    if (h->p.es == 8) advance2_t<double>(h, n);
    else advance2_t<float>(h, n);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail2(FDTD_E_DEVICE, "kernel launch failed: %s", hipGetErrorString(e));
    return FDTD_OK;
}

}  // namespace

extern "C" {

const char *fdtd2d_last_error(void) { return g_err2.c_str(); }

int fdtd2d_workspace_bytes(const fdtd2d_desc *desc, size_t *bytes)
{
    if (!bytes) return fail2(FDTD_E_INVALID, "bytes is NULL");
    Plan2 p;
    int rc = plan2(desc, p);
    if (rc) return rc;
    *bytes = (size_t)p.L.total;
    return FDTD_OK;
}

int fdtd2d_create(const fdtd2d_desc *desc, void *workspace, size_t bytes, fdtd2d **out)
{
    if (!out) return fail2(FDTD_E_INVALID, "out is NULL");
    *out = nullptr;
    fdtd2d *h = new (std::nothrow) fdtd2d();
    if (!h) return fail2(FDTD_E_INVALID, "out of host memory");
    int rc = plan2(desc, h->p);
    if (rc) {
        delete h;
        return rc;
    }
    Plan2 &p = h->p;
    if (workspace && (bytes < (size_t)p.L.total || ((uintptr_t)workspace % kAlign2))) {
        delete h;
        return fail2(FDTD_E_WORKSPACE, "workspace of %zu bytes (needs %lld, %lld-byte aligned)", bytes,
                     (long long)p.L.total, (long long)kAlign2);
    }
    h->d = *desc;
    h->stream = (hipStream_t)desc->stream;
    if (workspace) {
        h->ws = (char *)workspace;
    } else {
        hipError_t e = hipMalloc((void **)&h->ws, (size_t)p.L.total);
        if (e != hipSuccess) {
            delete h;
            return fail2(FDTD_E_DEVICE, "hipMalloc(%lld) failed: %s", (long long)p.L.total, hipGetErrorString(e));
        }
        h->owns = true;
    }
    char *w = h->ws;
    Grid2 &g = h->g;
    g = Grid2{};
    g.nx = desc->nx;
    g.ny = desc->ny;
    g.mode = desc->mode;
    g.px = desc->periodic_x != 0;
    g.py = desc->periodic_y != 0;
    g.dt = desc->dt;
    g.d = desc->d;
    g.ch = desc->dt / (mu0() * desc->d);
    g.ce = desc->dt / (kEps0 * desc->d);
    g.span = (const int2 *)(w + p.o_span);
    g.rowoff = (const int64_t *)(w + p.o_rowoff);
    for (int c = 0; c < 2; ++c) {
        const int cc = c < p.ncomp ? c : 0;
        g.wp2[c] = (const double *)(w + p.o_wp2[cc]);
        g.nu[c] = (const double *)(w + p.o_nu[cc]);
        g.J[c] = (double *)(w + p.o_J[cc]);
        h->E[c] = w + p.o_E[c < p.ncomp ? c : 0];
        h->H[c] = w + p.o_H[c < p.nh ? c : 0];
    }
    g.has_src = desc->has_src != 0;
    g.si = desc->src_i;
    g.sj = desc->src_j;
    g.src_tau = desc->src_tau;
    g.src_t0 = desc->src_t0;
    g.src_amp = desc->src_amp;
    g.P = desc->n_probes;
    g.SB = kSB2;
    g.probes = (const int64_t *)(w + p.o_probes);
    h->samp = g.samp = (double *)(w + p.o_samp);
    h->freqs = (double *)(w + p.o_freqs);
    h->X = (double2 *)(w + p.o_X);
    h->Xtmp = (double2 *)(w + p.o_Xtmp);
    h->tw = (double2 *)(w + p.o_tw);
    h->d.wp2 = h->d.nu = nullptr;
    h->d.probes = nullptr;
    h->d.freqs_hz = nullptr;

    // compact plasma arrays
    std::vector<double> cw(std::max<int64_t>(p.S, 1) * p.ncomp), cn(std::max<int64_t>(p.S, 1) * p.ncomp);
    for (int c = 0; c < p.ncomp; ++c)
        for (int64_t i = 0; i < desc->nx; ++i)
            for (int64_t j = p.span[i].x; j < p.span[i].y; ++j) {
                const int64_t src = c * p.N + i * desc->ny + j, dst = c * p.S + p.rowoff[i] + (j - p.span[i].x);
                cw[dst] = desc->wp2[src];
                cn[dst] = desc->nu[src];
            }
    hipStream_t st = h->stream;
    hipError_t e = hipSuccess;
    auto H2D = [&](void *dst, const void *src, size_t n) {
        if (e == hipSuccess && n) e = hipMemcpyAsync(dst, src, n, hipMemcpyHostToDevice, st);
    };
    H2D(w + p.o_span, p.span.data(), 8 * desc->nx);
    H2D(w + p.o_rowoff, p.rowoff.data(), 8 * desc->nx);
    for (int c = 0; c < p.ncomp; ++c) {
        H2D(w + p.o_wp2[c], cw.data() + c * p.S, 8 * p.S);
        H2D(w + p.o_nu[c], cn.data() + c * p.S, 8 * p.S);
    }
    if (desc->n_probes > 0) H2D(w + p.o_probes, desc->probes, 24 * (size_t)desc->n_probes);
    H2D(w + p.o_freqs, desc->freqs_hz, 8 * (size_t)desc->n_freqs);
    if (e == hipSuccess) {
        reset2(h);
        e = hipStreamSynchronize(st);
    }
    if (e == hipSuccess) e = hipGetLastError();
    if (e != hipSuccess) {
        if (h->owns) (void)hipFree(h->ws);
        delete h;
        return fail2(FDTD_E_DEVICE, "create failed: %s", hipGetErrorString(e));
    }
    *out = h;
    return FDTD_OK;
}

int fdtd2d_step(fdtd2d *h, int64_t nsteps)
{
    if (!h) return fail2(FDTD_E_INVALID, "handle is NULL");
    if (nsteps < 0) return fail2(FDTD_E_INVALID, "nsteps %lld < 0", (long long)nsteps);
    h->tmp_valid = false;
    return advance2(h, nsteps);
}

int fdtd2d_run(fdtd2d *h, int64_t nsteps)
{
    if (!h) return fail2(FDTD_E_INVALID, "handle is NULL");
    if (nsteps < 0) return fail2(FDTD_E_INVALID, "nsteps %lld < 0", (long long)nsteps);
    h->tmp_valid = false;
    if (h->stream == nullptr) {   // the legacy null stream cannot be captured
        reset2(h);
        int rc = advance2(h, nsteps);
        if (rc) return rc;
        to_tmp(h);
        h->tmp_valid = nsteps > 0;
        return FDTD_OK;
    }
    auto it = h->graphs.find(nsteps);
    if (it == h->graphs.end()) {
        HIP_TRY2(hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
        reset2(h);
        int rc = advance2(h, nsteps);
        if (rc == FDTD_OK) to_tmp(h);
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamEndCapture(h->stream, &graph);
        if (rc) {
            if (graph) (void)hipGraphDestroy(graph);
            return rc;
        }
        if (e != hipSuccess) return fail2(FDTD_E_DEVICE, "graph capture failed: %s", hipGetErrorString(e));
        hipGraphExec_t ex = nullptr;
        e = hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) return fail2(FDTD_E_DEVICE, "graph instantiate failed: %s", hipGetErrorString(e));
        it = h->graphs.emplace(nsteps, ex).first;
    } else {
        h->steps = nsteps;
        h->win_base = nsteps / kSB2 * kSB2;
    }
    HIP_TRY2(hipGraphLaunch(it->second, h->stream));
    h->tmp_valid = nsteps > 0;
    return FDTD_OK;
}

int fdtd2d_spectra(fdtd2d *h, double *re, double *im)
{
    if (!h) return fail2(FDTD_E_INVALID, "handle is NULL");
    if (!re || !im) return fail2(FDTD_E_INVALID, "output pointer is NULL");
    if (h->steps == 0 || h->d.n_probes == 0) return fail2(FDTD_E_STATE, "no step taken yet, or no probes");
    if (!h->tmp_valid) to_tmp(h);
    const int64_t n = (int64_t)h->d.n_probes * h->d.n_freqs;
    std::vector<double2> X(n);
    HIP_TRY2(hipMemcpyAsync(X.data(), h->Xtmp, 16 * n, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY2(hipStreamSynchronize(h->stream));
    bool finite = true;
    for (int64_t i = 0; i < n; ++i) {
        re[i] = X[i].x;
        im[i] = X[i].y;
        finite = finite && std::isfinite(X[i].x) && std::isfinite(X[i].y);
    }
    return finite ? FDTD_OK : fail2(FDTD_E_NONFINITE, "a probe spectrum holds NaN or Inf");
}

int fdtd2d_get_fields(fdtd2d *h, int32_t which, double *out)
{
    if (!h) return fail2(FDTD_E_INVALID, "handle is NULL");
    if (!out) return fail2(FDTD_E_INVALID, "output pointer is NULL");
    const Plan2 &p = h->p;
    if (which < 0 || which >= 2 * p.ncomp + p.nh) return fail2(FDTD_E_INVALID, "which %d out of range", which);
    const int64_t N = p.N;
    if (which < p.ncomp + p.nh) {
        const void *src = which < p.ncomp ? h->E[which] : h->H[which - p.ncomp];
        std::vector<char> buf(p.es * N);
        HIP_TRY2(hipMemcpyAsync(buf.data(), src, p.es * N, hipMemcpyDeviceToHost, h->stream));
        HIP_TRY2(hipStreamSynchronize(h->stream));
        for (int64_t k = 0; k < N; ++k)
            out[k] = p.es == 8 ? ((const double *)buf.data())[k] : (double)((const float *)buf.data())[k];
        return FDTD_OK;
    }
    const int c = which - p.ncomp - p.nh;
    std::vector<double> Jc(std::max<int64_t>(p.S, 1));
    if (p.S) {
        HIP_TRY2(hipMemcpyAsync(Jc.data(), h->g.J[c], 8 * p.S, hipMemcpyDeviceToHost, h->stream));
        HIP_TRY2(hipStreamSynchronize(h->stream));
    }
    std::memset(out, 0, 8 * N);
    for (int64_t i = 0; i < h->d.nx; ++i)
        for (int64_t j = p.span[i].x; j < p.span[i].y; ++j) out[i * h->d.ny + j] = Jc[p.rowoff[i] + j - p.span[i].x];
    return FDTD_OK;
}

int fdtd2d_steps_done(fdtd2d *h, int64_t *steps)
{
    if (!h || !steps) return fail2(FDTD_E_INVALID, "NULL argument");
    *steps = h->steps;
    return FDTD_OK;
}

int fdtd2d_destroy(fdtd2d *h)
{
    if (!h) return FDTD_OK;
    (void)hipStreamSynchronize(h->stream);
    for (auto &kv : h->graphs) (void)hipGraphExecDestroy(kv.second);
    if (h->owns && h->ws) (void)hipFree(h->ws);
    delete h;
    return FDTD_OK;
}

}  // extern "C"
