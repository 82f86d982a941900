// C-ABI of the 3D library (fdtd_plasma3d.h): validation, workspace layout,
// plasma-support compaction, CPML tables, the time loop (eager or as a
// captured hipGraph), DFT buffering and field I/O.  Every step of the method
// runs in kernels3d.hip; the host builds index tables and launches.
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

#include "../../include/fdtd_plasma3d.h"
#include "internal3d.h"

using namespace fdtdp;

namespace {

thread_local std::string g_err3;

int fail3(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err3 = buf;
    return code;
}

#define HIP3(expr)                                                                          \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail3(FDTD_E_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));    \
    } while (0)

constexpr int64_t kAlign3 = 256;
constexpr int kAuxMargin = 8;      // incident grid spans z in [tf_lo - 8, tf_hi + 8]
constexpr int kAuxSrc = 3;         // its soft source node (z = tf_lo - 5)

int64_t up3(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

struct Layout3 {
    int64_t total = 0;
    int64_t take(int64_t bytes)
    {
        const int64_t o = total;
        total += up3(std::max<int64_t>(bytes, 16), kAlign3);
        return o;
    }
};

// Everything create needs to know before allocating.
struct Plan3 {
    int64_t N = 0, rows = 0, S = 0;       // cells, rows (i, j), compact support size
    int esize = 8;
    int K = 32;                           // sample slots
    int64_t npts = 0;
    int F = 0;
    int P = 0;
    int64_t na = 1, ao = 0;               // incident grid nodes and z = 0 node
    int64_t slab[3] = {0, 0, 0};          // CPML slab array sizes per axis (0: none)
    std::vector<int2> span;               // per row
    std::vector<int64_t> off;
    int exec = FDTD3D_EXEC_FUSED;
    int ni = 32;                          // planes per fused-kernel chunk
    // workspace offsets; [2]: the two copies of the ping-ponged state
    int64_t oE[2][3], oH[2][3], oJ[3], oW[3], oNu[3], oSpan, oOff, oPsiH[2][3][2], oPsiE[2][3][2], oTab,
        oEi[2], oHi, oPts, oFreq, oX, oXt, oBuf, oTw;
    int64_t oCA[3], oCJ[3], oCH[3], oCa[3], oCb1[3], oCb2[3];   // coefficient tables of the support
    int64_t total = 0;
};

int validate3(const fdtd3d_desc *d)
{
    if (!d) return fail3(FDTD_E_INVALID, "desc is NULL");
    if (d->struct_size != (int32_t)sizeof(fdtd3d_desc))
        return fail3(FDTD_E_INVALID, "struct_size %d, expected %d", d->struct_size, (int)sizeof(fdtd3d_desc));
    if (d->precision != FDTD_F64 && d->precision != FDTD_F32)
        return fail3(FDTD_E_INVALID, "precision %d", d->precision);
    if (d->nx < 2 || d->ny < 2 || d->nz < 4)
        return fail3(FDTD_E_INVALID, "grid %lld x %lld x %lld (need >= 2 x 2 x 4)", (long long)d->nx,
                     (long long)d->ny, (long long)d->nz);
    const double N = (double)d->nx * (double)d->ny * (double)d->nz;
    if (N > 4.0e9 || (double)d->nx * (double)d->ny > 2.0e9)
        return fail3(FDTD_E_INVALID, "grid too large");
    if (!(d->d > 0.0) || !(d->dt > 0.0) || !std::isfinite(d->d) || !std::isfinite(d->dt))
        return fail3(FDTD_E_INVALID, "d and dt must be positive");
    if (kC0 * d->dt / d->d > 1.0 / std::sqrt(3.0))
        return fail3(FDTD_E_UNSTABLE, "Courant number c dt/d = %.6g above 1/sqrt(3)", kC0 * d->dt / d->d);
    if (d->periodic_x < 0 || d->periodic_x > 1 || d->periodic_y < 0 || d->periodic_y > 1)
        return fail3(FDTD_E_INVALID, "periodic flags must be 0 or 1");
    const int P = d->cpml_cells;
    if (P < 0 || 2LL * P >= d->nz || (P > 0 && ((!d->periodic_x && 2LL * P >= d->nx) ||
                                                (!d->periodic_y && 2LL * P >= d->ny))))
        return fail3(FDTD_E_INVALID, "cpml_cells %d does not fit the walled axes", P);
    for (int c = 0; c < 3; ++c)
        if (!d->wp2[c] || !d->nu[c]) return fail3(FDTD_E_INVALID, "wp2[%d] / nu[%d] is NULL", c, c);
    if (d->source < FDTD3D_SRC_NONE || d->source > FDTD3D_SRC_TFSF)
        return fail3(FDTD_E_INVALID, "source %d", d->source);
    if (d->source == FDTD3D_SRC_PLANAR &&
        (d->src_comp < 0 || d->src_comp > 1 || d->src_k < 0 || d->src_k >= d->nz))
        return fail3(FDTD_E_INVALID, "planar source component %d plane %lld", d->src_comp, (long long)d->src_k);
    if (d->source == FDTD3D_SRC_TFSF) {
        const int64_t b0 = d->tf_lo, b1 = d->tf_hi;
        bool ok = b0 >= 1 && b1 > b0 && b1 <= d->nz - 1;
        if (!d->periodic_x) ok = ok && b1 <= d->nx - 1;
        if (!d->periodic_y) ok = ok && b1 <= d->ny - 1;
        if (!ok) return fail3(FDTD_E_INVALID, "TF box [%lld, %lld] outside the grid", (long long)b0, (long long)b1);
    }
    if (d->source != FDTD3D_SRC_NONE && !(d->src_tau > 0.0))
        return fail3(FDTD_E_INVALID, "src_tau must be positive");
    if (d->n_points < 0 || d->n_freqs < 0) return fail3(FDTD_E_INVALID, "negative n_points / n_freqs");
    if (d->n_points > 0 && !d->points) return fail3(FDTD_E_INVALID, "points is NULL");
    if (d->n_freqs > 0 && !d->freqs_hz) return fail3(FDTD_E_INVALID, "freqs_hz is NULL");
    for (int32_t q = 0; q < d->n_points; ++q) {
        const int32_t *s = d->points + 4 * (int64_t)q;
        if (s[0] < 0 || s[0] > 5 || s[1] < 0 || s[1] >= d->nx || s[2] < 0 || s[2] >= d->ny || s[3] < 0 ||
            s[3] >= d->nz)
            return fail3(FDTD_E_INVALID, "sample point %d (%d, %d, %d, %d) out of range", q, s[0], s[1], s[2], s[3]);
    }
    for (int32_t f = 0; f < d->n_freqs; ++f)
        if (!std::isfinite(d->freqs_hz[f])) return fail3(FDTD_E_INVALID, "freqs_hz[%d] not finite", f);
    if (d->sample_slots < 0 || d->sample_slots > kSlotsMax)
        return fail3(FDTD_E_INVALID, "sample_slots %d (0..%d)", d->sample_slots, kSlotsMax);
    if (d->exec < FDTD3D_EXEC_AUTO || d->exec > FDTD3D_EXEC_FUSED)
        return fail3(FDTD_E_INVALID, "exec %d", d->exec);
    const bool fused = d->exec == FDTD3D_EXEC_FUSED;
    if (d->x_planes != 0 && (fused ? (d->x_planes < 2 || d->x_planes > 128) : (d->x_planes < 1 || d->x_planes > 16)))
        return fail3(FDTD_E_INVALID, "x_planes %d out of range for this executor", d->x_planes);
    return FDTD_OK;
}

// Scan the plasma support and lay out the workspace.
int plan3(const fdtd3d_desc *d, Plan3 &pl, bool keep_tables)
{
    int rc = validate3(d);
    if (rc) return rc;
    pl.N = d->nx * d->ny * d->nz;
    pl.rows = d->nx * d->ny;
    pl.esize = d->precision == FDTD_F64 ? 8 : 4;
    pl.K = d->sample_slots ? d->sample_slots : 32;
    pl.npts = d->n_points;
    pl.F = d->n_freqs;
    pl.P = d->cpml_cells;
    const int64_t nz = d->nz;
    if (keep_tables) {
        pl.span.assign(pl.rows, make_int2(0, 0));
        pl.off.assign(pl.rows, 0);
    }
    int64_t S = 0;
    for (int64_t r = 0; r < pl.rows; ++r) {
        int64_t k0 = nz, k1 = 0;
        for (int c = 0; c < 3; ++c) {
            const double *w = d->wp2[c] + r * nz, *v = d->nu[c] + r * nz;
            for (int64_t k = 0; k < nz; ++k) {
                if (!(w[k] >= 0.0) || !std::isfinite(w[k]) || !(v[k] >= 0.0) || !std::isfinite(v[k]))
                    return fail3(FDTD_E_INVALID, "wp2/nu of component %d at node %lld invalid", c,
                                 (long long)(r * nz + k));
                if (w[k] > 0.0) {
                    k0 = std::min(k0, k);
                    k1 = std::max(k1, k + 1);
                }
            }
        }
        if (k1 > k0) {
            if (keep_tables) {
                pl.span[r] = make_int2((int)k0, (int)k1);
                pl.off[r] = S;
            }
            S += k1 - k0;
        }
    }
    pl.S = S;
    if (d->source == FDTD3D_SRC_TFSF) {
        pl.na = d->tf_hi - d->tf_lo + 2 * kAuxMargin + 1;
        pl.ao = kAuxMargin - d->tf_lo;
    }
    const int64_t P2 = 2LL * pl.P;
    if (pl.P > 0) {
        pl.slab[0] = d->periodic_x ? 0 : P2 * d->ny * d->nz;
        pl.slab[1] = d->periodic_y ? 0 : d->nx * P2 * d->nz;
        pl.slab[2] = d->nx * d->ny * P2;
    }
    pl.exec = d->exec == FDTD3D_EXEC_FUSED ? FDTD3D_EXEC_FUSED : FDTD3D_EXEC_SPLIT;
    // the fused kernel's x chunks: enough workgroups to fill 256 CUs several
    // times over, chunks long enough that the one-plane lead-in stays small;
    // the split kernels' planes per thread
    pl.ni = d->x_planes ? d->x_planes : (pl.exec == FDTD3D_EXEC_FUSED ? 32 : 4);
    Layout3 L;
    const int es = pl.esize;
    const int copies = pl.exec == FDTD3D_EXEC_FUSED ? 2 : 1;
    for (int cp = 0; cp < 2; ++cp)
        for (int c = 0; c < 3; ++c) {
            pl.oE[cp][c] = cp < copies ? L.take(pl.N * es) : pl.oE[0][c];
            pl.oH[cp][c] = cp < copies ? L.take(pl.N * es) : pl.oH[0][c];
        }
    for (int c = 0; c < 3; ++c) pl.oJ[c] = L.take(S * es);
    for (int cp = 0; cp < 2; ++cp)
        for (int a = 0; a < 3; ++a)
            for (int q = 0; q < 2; ++q) {
                const bool have = pl.slab[a] && cp < copies;
                pl.oPsiH[cp][a][q] = have ? L.take(pl.slab[a] * es) : (pl.slab[a] ? pl.oPsiH[0][a][q] : -1);
                pl.oPsiE[cp][a][q] = have ? L.take(pl.slab[a] * es) : (pl.slab[a] ? pl.oPsiE[0][a][q] : -1);
            }
    pl.oEi[0] = L.take(pl.na * 8);
    pl.oEi[1] = L.take(pl.na * 8);
    pl.oHi = L.take(pl.na * 8);
    pl.oX = L.take(pl.npts * pl.F * 16);
    // (above: the state that a reset zeroes; below: tables and scratch)
    for (int c = 0; c < 3; ++c) pl.oW[c] = L.take(S * 8);
    for (int c = 0; c < 3; ++c) pl.oNu[c] = L.take(S * 8);
    for (int c = 0; c < 3; ++c) {
        pl.oCA[c] = L.take(S * es);
        pl.oCJ[c] = L.take(S * es);
        pl.oCH[c] = L.take(S * es);
        pl.oCa[c] = L.take(S * es);
        pl.oCb1[c] = L.take(S * es);
        pl.oCb2[c] = L.take(S * es);
    }
    pl.oSpan = L.take(pl.rows * 8);
    pl.oOff = L.take(pl.rows * 8);
    pl.oTab = L.take(3 * 4 * std::max<int64_t>(P2, 1) * es);
    pl.oPts = L.take(pl.npts * 8);
    pl.oFreq = L.take(pl.F * 8);
    pl.oXt = L.take(pl.npts * pl.F * 16);
    pl.oBuf = L.take((int64_t)pl.K * pl.npts * es);
    pl.oTw = L.take(2LL * pl.K * pl.F * 16);
    pl.total = L.total;
    return FDTD_OK;
}

// CPML depth of a position on an axis of n cells (walls at 0 and n)
double depth_of(int64_t n, int P, double pos)
{
    if (pos < (double)P) return (double)P - pos;
    if (pos > (double)(n - P)) return pos - (double)(n - P);
    return 0.0;
}

}  // namespace

struct ProfRec3 {
    int kind;
    hipEvent_t a, b;
    double cells;
};

struct fdtd3d {
    fdtd3d_desc d{};
    Plan3 pl;
    hipStream_t stream = nullptr;
    int device = 0;
    bool owns_ws = false;
    char *ws = nullptr;
    Geo3 geo{};
    double cm = 0.0;
    int64_t asrc = kAuxSrc;
    std::vector<double> freqs;
    int64_t steps = 0;
    int cur = 0;              // copy holding the state (fused executor)
    int acur = 0;             // incident-grid E copy holding Einc^n
    int slot = 0;
    int64_t win_base = 0;
    std::map<int64_t, hipGraphExec_t> graphs;
    bool prof = false;
    std::vector<ProfRec3> recs;
    bool poisoned = false;

    template <typename T>
    T *at(int64_t o) const { return o < 0 ? nullptr : (T *)(ws + o); }
};

namespace {

constexpr int kKinds = 6;
const char *kProfNames[kKinds] = {"k_h3d", "k_aux3d", "k_e3d", "k_sample3d", "k_tw3d+k_flush3d", "k_fused3d"};

template <typename T>
Fields3<T> fields_of(const fdtd3d *h, int cp)
{
    Fields3<T> f;
    for (int c = 0; c < 3; ++c) {
        f.E[c] = h->at<T>(h->pl.oE[cp][c]);
        f.H[c] = h->at<T>(h->pl.oH[cp][c]);
    }
    return f;
}

// CPML auxiliaries read from copy `in` and written to copy `out`
template <typename T>
Cpml3<T> cpml_of(const fdtd3d *h, int in, int out)
{
    Cpml3<T> c;
    for (int a = 0; a < 3; ++a)
        for (int q = 0; q < 2; ++q) {
            c.inH[a][q] = h->at<T>(h->pl.oPsiH[in][a][q]);
            c.outH[a][q] = h->at<T>(h->pl.oPsiH[out][a][q]);
            c.inE[a][q] = h->at<T>(h->pl.oPsiE[in][a][q]);
            c.outE[a][q] = h->at<T>(h->pl.oPsiE[out][a][q]);
        }
    c.tab = h->at<T>(h->pl.oTab);
    return c;
}

template <typename T>
Plasma3<T> plasma_of(const fdtd3d *h)
{
    Plasma3<T> p;
    p.span = h->at<int2>(h->pl.oSpan);
    p.off = h->at<int64_t>(h->pl.oOff);
    for (int c = 0; c < 3; ++c) {
        p.J[c] = h->at<T>(h->pl.oJ[c]);
        p.eA[c] = h->at<T>(h->pl.oCA[c]);
        p.eJ[c] = h->at<T>(h->pl.oCJ[c]);
        p.eH[c] = h->at<T>(h->pl.oCH[c]);
        p.ca[c] = h->at<T>(h->pl.oCa[c]);
        p.cb1[c] = h->at<T>(h->pl.oCb1[c]);
        p.cb2[c] = h->at<T>(h->pl.oCb2[c]);
    }
    return p;
}

void prof_begin(fdtd3d *h, int kind, double cells, ProfRec3 &r)
{
    r.kind = kind;
    r.cells = cells;
    r.a = r.b = nullptr;
    if (!h->prof) return;
    (void)hipEventCreate(&r.a);
    (void)hipEventCreate(&r.b);
    (void)hipEventRecord(r.a, h->stream);
}

void prof_end(fdtd3d *h, ProfRec3 &r)
{
    if (!h->prof) return;
    (void)hipEventRecord(r.b, h->stream);
    h->recs.push_back(r);
}

// zero the state regions (E, H, J, psi, incident grid, accumulators): they are
// laid out first and contiguously
void reset3(fdtd3d *h)
{
    launch_fill3d(h->ws, up3(h->pl.oX + h->pl.npts * h->pl.F * 16, 16), h->stream);
    h->steps = 0;
    h->cur = 0;
    h->acur = 0;
    h->slot = 0;
    h->win_base = 0;
}

template <typename T>
void one_step(fdtd3d *h)
{
    const int cur = h->cur, nxt = h->pl.exec == FDTD3D_EXEC_FUSED ? cur ^ 1 : cur;
    const Fields3<T> f = fields_of<T>(h, cur);
    const Cpml3<T> c = cpml_of<T>(h, cur, nxt);
    const Plasma3<T> p = plasma_of<T>(h);
    const double tnew = (double)(h->steps + 1) * h->d.dt;
    const double s = h->d.source != FDTD3D_SRC_NONE
                         ? source_value(tnew, h->d.src_tau, h->d.src_t0, h->d.src_amp)
                         : 0.0;
    const bool tfsf = h->d.source == FDTD3D_SRC_TFSF;
    const double *Ei = h->at<double>(h->pl.oEi[h->acur]);
    double *Eo = h->at<double>(h->pl.oEi[h->acur ^ 1]), *Hi = h->at<double>(h->pl.oHi);
    const double cells = (double)h->pl.N;
    ProfRec3 r;
    if (h->pl.exec == FDTD3D_EXEC_FUSED) {
        if (tfsf) {
            prof_begin(h, 1, (double)h->pl.na, r);
            launch_aux3d(Ei, Eo, Hi, h->pl.na, h->asrc, h->geo.chd, h->geo.ced, h->cm, s, h->stream);
            prof_end(h, r);
        }
        prof_begin(h, 5, cells, r);
        launch_fused3d<T>(h->geo, f, fields_of<T>(h, nxt), p, c, Ei, Hi, s, h->pl.ni, h->stream);
        prof_end(h, r);
    } else {
        prof_begin(h, 0, cells, r);
        launch_h3d<T>(h->geo, f, c, Ei, h->stream);
        prof_end(h, r);
        if (tfsf) {
            prof_begin(h, 1, (double)h->pl.na, r);
            launch_aux3d(Ei, Eo, Hi, h->pl.na, h->asrc, h->geo.chd, h->geo.ced, h->cm, s, h->stream);
            prof_end(h, r);
        }
        prof_begin(h, 2, cells, r);
        launch_e3d<T>(h->geo, f, p, c, Hi, s, h->stream);
        prof_end(h, r);
    }
    if (tfsf) h->acur ^= 1;
    h->cur = nxt;
    h->steps += 1;
    if (h->pl.npts > 0 && h->pl.F > 0) {
        T *buf = h->at<T>(h->pl.oBuf) + (int64_t)h->slot * h->pl.npts;
        prof_begin(h, 3, (double)h->pl.npts, r);
        launch_sample3d<T>(fields_of<T>(h, h->cur), h->pl.N, h->at<int64_t>(h->pl.oPts), h->pl.npts, buf,
                           h->stream);
        prof_end(h, r);
        h->slot += 1;
        if (h->slot == h->pl.K) {
            prof_begin(h, 4, (double)h->pl.npts * h->pl.F * h->pl.K, r);
            launch_tw3d(h->at<double>(h->pl.oFreq), h->pl.F, h->d.dt, h->win_base, h->pl.K,
                        h->at<double2>(h->pl.oTw), h->stream);
            launch_flush3d<T>(h->at<T>(h->pl.oBuf), h->pl.K, h->pl.npts, h->at<int64_t>(h->pl.oPts), h->pl.N,
                              h->pl.F, h->at<double2>(h->pl.oTw), h->at<double2>(h->pl.oX), h->stream);
            prof_end(h, r);
            h->win_base += h->pl.K;
            h->slot = 0;
        }
    }
}

int advance3(fdtd3d *h, int64_t nsteps)
{
    for (int64_t s = 0; s < nsteps; ++s) {
        if (h->pl.esize == 8) one_step<double>(h);
        else one_step<float>(h);
    }
    HIP3(hipGetLastError());
    return FDTD_OK;
}

int check3(fdtd3d *h)
{
    if (!h) return fail3(FDTD_E_INVALID, "handle is NULL");
    if (h->poisoned) return fail3(FDTD_E_STATE, "handle unusable after a failed capture");
    HIP3(hipSetDevice(h->device));
    return FDTD_OK;
}

}  // namespace

extern "C" {

int fdtd3d_workspace_bytes(const fdtd3d_desc *desc, size_t *bytes)
{
    if (!bytes) return fail3(FDTD_E_INVALID, "bytes is NULL");
    Plan3 pl;
    int rc = plan3(desc, pl, false);
    if (rc) return rc;
    *bytes = (size_t)pl.total;
    return FDTD_OK;
}

int fdtd3d_create(const fdtd3d_desc *desc, void *workspace, size_t bytes, fdtd3d **out)
{
    if (!out) return fail3(FDTD_E_INVALID, "out is NULL");
    *out = nullptr;
    fdtd3d *h = new (std::nothrow) fdtd3d();
    if (!h) return fail3(FDTD_E_INVALID, "out of host memory");
    auto undo = [&](int rc) {
        if (h->owns_ws && h->ws) (void)hipFree(h->ws);
        delete h;
        return rc;
    };
    int rc = plan3(desc, h->pl, true);
    if (rc) return undo(rc);
    h->d = *desc;
    h->stream = (hipStream_t)desc->stream;
    if (hipGetDevice(&h->device) != hipSuccess)
        return undo(fail3(FDTD_E_DEVICE, "no HIP device: %s", hipGetErrorString(hipGetLastError())));
    const Plan3 &pl = h->pl;
    if (workspace) {
        if ((size_t)pl.total > bytes) return undo(fail3(FDTD_E_WORKSPACE, "workspace %zu bytes, need %lld", bytes, (long long)pl.total));
        if (((uintptr_t)workspace) % kAlign3) return undo(fail3(FDTD_E_WORKSPACE, "workspace not 256-byte aligned"));
        h->ws = (char *)workspace;
    } else {
        hipError_t e = hipMalloc((void **)&h->ws, (size_t)pl.total);
        if (e != hipSuccess) {
            h->ws = nullptr;
            return undo(fail3(FDTD_E_DEVICE, "hipMalloc(%lld) failed: %s", (long long)pl.total, hipGetErrorString(e)));
        }
        h->owns_ws = true;
    }
    const fdtd3d_desc &d = h->d;
    // geometry
    Geo3 &g = h->geo;
    g.nx = d.nx;
    g.ny = d.ny;
    g.nz = d.nz;
    g.kb = (d.nz + 63) / 64;
    g.np = pl.exec == FDTD3D_EXEC_FUSED ? 1 : pl.ni;
    g.jb = (d.ny + 3) / 4;
    g.px = d.periodic_x;
    g.py = d.periodic_y;
    g.P = d.cpml_cells;
    g.src = d.source;
    g.src_comp = d.src_comp;
    g.src_k = d.src_k;
    g.b0 = d.tf_lo;
    g.b1 = d.tf_hi;
    g.xlo = d.periodic_x ? 0 : d.tf_lo;
    g.xhi = d.periodic_x ? d.nx : d.tf_hi;
    g.ylo = d.periodic_y ? 0 : d.tf_lo;
    g.yhi = d.periodic_y ? d.ny : d.tf_hi + 1;
    g.ao = pl.ao;
    g.chd = d.dt / (mu0() * d.d);
    g.ced = d.dt / (kEps0 * d.d);
    g.dt = d.dt;
    g.d = d.d;
    const double S = kC0 * d.dt / d.d;
    h->cm = (S - 1.0) / (S + 1.0);
    if (g.kb * g.jb * g.nx > 0x7fffffffLL) return undo(fail3(FDTD_E_INVALID, "grid needs too many workgroups"));
    // host tables
    std::vector<double> wc(pl.S), nc(pl.S);
    hipError_t e = hipSuccess;
    for (int c = 0; c < 3 && e == hipSuccess; ++c) {
        for (int64_t r = 0; r < pl.rows; ++r) {
            const int2 sp = pl.span[r];
            for (int k = sp.x; k < sp.y; ++k) {
                wc[pl.off[r] + (k - sp.x)] = d.wp2[c][r * d.nz + k];
                nc[pl.off[r] + (k - sp.x)] = d.nu[c][r * d.nz + k];
            }
        }
        if (pl.S > 0) e = hipMemcpy(h->ws + pl.oW[c], wc.data(), pl.S * 8, hipMemcpyHostToDevice);
        if (e == hipSuccess && pl.S > 0) e = hipMemcpy(h->ws + pl.oNu[c], nc.data(), pl.S * 8, hipMemcpyHostToDevice);
    }
    if (e == hipSuccess) e = hipMemcpy(h->ws + pl.oSpan, pl.span.data(), pl.rows * 8, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(h->ws + pl.oOff, pl.off.data(), pl.rows * 8, hipMemcpyHostToDevice);
    // CPML tables by slab index: the same grading as the 1D library
    if (e == hipSuccess && pl.P > 0) {
        const int P = pl.P, P2 = 2 * P;
        const double m = 3.0, eta0 = std::sqrt(mu0() / kEps0), smax = 0.8 * (m + 1.0) / (eta0 * d.d);
        std::vector<double> tab(3 * 4 * P2);
        const int64_t len[3] = {d.nx, d.ny, d.nz};
        for (int a = 0; a < 3; ++a)
            for (int s = 0; s < P2; ++s) {
                const int64_t node = s < P ? s : len[a] - P2 + s;
                for (int kind = 0; kind < 2; ++kind) {       // 0: E (integer), 1: H (half-integer)
                    const double depth = depth_of(len[a], P, (double)node + (kind ? 0.5 : 0.0));
                    double b = 1.0, aa = 0.0;
                    if (depth > 0.0) {
                        const double sigma = smax * std::pow(depth / (double)P, m);
                        b = std::exp(-sigma * d.dt / kEps0);
                        aa = b - 1.0;
                    }
                    tab[(a * 4 + 2 * kind) * P2 + s] = b;
                    tab[(a * 4 + 2 * kind + 1) * P2 + s] = aa;
                }
            }
        if (pl.esize == 8) {
            e = hipMemcpy(h->ws + pl.oTab, tab.data(), tab.size() * 8, hipMemcpyHostToDevice);
        } else {
            std::vector<float> tf(tab.begin(), tab.end());
            e = hipMemcpy(h->ws + pl.oTab, tf.data(), tf.size() * 4, hipMemcpyHostToDevice);
        }
    }
    if (e == hipSuccess && pl.npts > 0) {
        std::vector<int64_t> codes(pl.npts);
        for (int64_t q = 0; q < pl.npts; ++q) {
            const int32_t *s = d.points + 4 * q;
            codes[q] = (int64_t)s[0] * pl.N + ((int64_t)s[1] * d.ny + s[2]) * d.nz + s[3];
        }
        e = hipMemcpy(h->ws + pl.oPts, codes.data(), pl.npts * 8, hipMemcpyHostToDevice);
    }
    if (e == hipSuccess && pl.F > 0) {
        h->freqs.assign(d.freqs_hz, d.freqs_hz + pl.F);
        e = hipMemcpy(h->ws + pl.oFreq, h->freqs.data(), pl.F * 8, hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) return undo(fail3(FDTD_E_DEVICE, "create copies failed: %s", hipGetErrorString(e)));
    // coefficient tables of the plasma support (a0), built on the device
    if (e == hipSuccess && pl.S > 0) {
        const double *w[3], *n[3];
        void *eA[3], *eJ[3], *eH[3], *ca[3], *cb1[3], *cb2[3];
        for (int c = 0; c < 3; ++c) {
            w[c] = h->at<double>(pl.oW[c]);
            n[c] = h->at<double>(pl.oNu[c]);
            ca[c] = h->ws + pl.oCa[c];
            cb1[c] = h->ws + pl.oCb1[c];
            cb2[c] = h->ws + pl.oCb2[c];
            eA[c] = h->ws + pl.oCA[c];
            eJ[c] = h->ws + pl.oCJ[c];
            eH[c] = h->ws + pl.oCH[c];
        }
        if (pl.esize == 8)
            launch_coef3d<double>(w, n, pl.S, d.dt, d.d, (double *const *)eA, (double *const *)eJ,
                                  (double *const *)eH, (double *const *)ca, (double *const *)cb1,
                                  (double *const *)cb2, h->stream);
        else
            launch_coef3d<float>(w, n, pl.S, d.dt, d.d, (float *const *)eA, (float *const *)eJ,
                                 (float *const *)eH, (float *const *)ca, (float *const *)cb1,
                                 (float *const *)cb2, h->stream);
        e = hipGetLastError();
    }
    // the host pointers of the caller are not kept
    for (int c = 0; c < 3; ++c) h->d.wp2[c] = h->d.nu[c] = nullptr;
    h->d.points = nullptr;
    h->d.freqs_hz = nullptr;
    reset3(h);
    e = hipStreamSynchronize(h->stream);
    if (e == hipSuccess) e = hipGetLastError();
    if (e != hipSuccess) return undo(fail3(FDTD_E_DEVICE, "create failed: %s", hipGetErrorString(e)));
    *out = h;
    return FDTD_OK;
}

int fdtd3d_step(fdtd3d *h, int64_t nsteps)
{
    int rc = check3(h);
    if (rc) return rc;
    if (nsteps < 0) return fail3(FDTD_E_INVALID, "nsteps %lld < 0", (long long)nsteps);
    return advance3(h, nsteps);
}

int fdtd3d_run(fdtd3d *h, int64_t nsteps)
{
    int rc = check3(h);
    if (rc) return rc;
    if (nsteps < 0) return fail3(FDTD_E_INVALID, "nsteps %lld < 0", (long long)nsteps);
    if (h->stream == nullptr || h->prof) {
        reset3(h);
        return advance3(h, nsteps);
    }
    auto it = h->graphs.find(nsteps);
    if (it == h->graphs.end()) {
        HIP3(hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
        reset3(h);
        rc = advance3(h, nsteps);
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamEndCapture(h->stream, &graph);
        if (rc || e != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            h->poisoned = true;
            return rc ? rc : fail3(FDTD_E_DEVICE, "graph capture failed: %s", hipGetErrorString(e));
        }
        hipGraphExec_t exec = nullptr;
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) return fail3(FDTD_E_DEVICE, "graph instantiate failed: %s", hipGetErrorString(e));
        it = h->graphs.emplace(nsteps, exec).first;
    } else {
        // bookkeeping of the captured launches
        h->steps = nsteps;
        h->cur = h->pl.exec == FDTD3D_EXEC_FUSED ? (int)(nsteps & 1) : 0;
        h->acur = h->d.source == FDTD3D_SRC_TFSF ? (int)(nsteps & 1) : 0;
        if (h->pl.npts > 0 && h->pl.F > 0) {
            h->slot = (int)(nsteps % h->pl.K);
            h->win_base = nsteps - h->slot;
        }
    }
    HIP3(hipGraphLaunch(it->second, h->stream));
    return FDTD_OK;
}

int fdtd3d_spectra(fdtd3d *h, double *re, double *im)
{
    int rc = check3(h);
    if (rc) return rc;
    if (!re || !im) return fail3(FDTD_E_INVALID, "re / im is NULL");
    const Plan3 &pl = h->pl;
    const int64_t n = pl.npts * pl.F;
    if (n == 0) return FDTD_OK;
    double2 *src = h->at<double2>(pl.oX);
    if (h->slot > 0) {
        // fold the buffered samples into a copy, leaving X and the window alone
        double2 *Xt = h->at<double2>(pl.oXt);
        launch_copy3d(Xt, src, n * 16, h->stream);
        launch_tw3d(h->at<double>(pl.oFreq), pl.F, h->d.dt, h->win_base, h->slot, h->at<double2>(pl.oTw), h->stream);
        if (pl.esize == 8)
            launch_flush3d<double>(h->at<double>(pl.oBuf), h->slot, pl.npts, h->at<int64_t>(pl.oPts), pl.N, pl.F,
                                   h->at<double2>(pl.oTw), Xt, h->stream);
        else
            launch_flush3d<float>(h->at<float>(pl.oBuf), h->slot, pl.npts, h->at<int64_t>(pl.oPts), pl.N, pl.F,
                                  h->at<double2>(pl.oTw), Xt, h->stream);
        src = Xt;
    }
    std::vector<double2> hx(n);
    HIP3(hipMemcpyAsync(hx.data(), src, n * 16, hipMemcpyDeviceToHost, h->stream));
    HIP3(hipStreamSynchronize(h->stream));
    bool finite = true;
    for (int64_t q = 0; q < pl.npts; ++q)
        for (int f = 0; f < pl.F; ++f) {
            const double2 x = hx[(int64_t)f * pl.npts + q];
            re[q * pl.F + f] = x.x;
            im[q * pl.F + f] = x.y;
            finite = finite && std::isfinite(x.x) && std::isfinite(x.y);
        }
    if (!finite) return fail3(FDTD_E_NONFINITE, "a spectrum entry is NaN or Inf");
    return FDTD_OK;
}

static int fields_io(fdtd3d *h, int32_t which, void *host, bool get)
{
    int rc = check3(h);
    if (rc) return rc;
    if (!host) return fail3(FDTD_E_INVALID, "host pointer is NULL");
    if (which < FDTD3D_EX || which > FDTD3D_JZ) return fail3(FDTD_E_INVALID, "field %d", which);
    const Plan3 &pl = h->pl;
    const int es = pl.esize;
    HIP3(hipStreamSynchronize(h->stream));
    if (which <= FDTD3D_HZ) {
        const int64_t o = which < 3 ? pl.oE[h->cur][which] : pl.oH[h->cur][which - 3];
        if (get) HIP3(hipMemcpy(host, h->ws + o, pl.N * es, hipMemcpyDeviceToHost));
        else HIP3(hipMemcpy(h->ws + o, host, pl.N * es, hipMemcpyHostToDevice));
        return FDTD_OK;
    }
    const int c = which - FDTD3D_JX;
    std::vector<char> comp(std::max<int64_t>(pl.S, 1) * es);
    char *hb = (char *)host;
    const int64_t nz = h->d.nz;
    if (get) {
        if (pl.S > 0) HIP3(hipMemcpy(comp.data(), h->ws + pl.oJ[c], pl.S * es, hipMemcpyDeviceToHost));
        memset(hb, 0, pl.N * es);
        for (int64_t r = 0; r < pl.rows; ++r) {
            const int2 sp = pl.span[r];
            if (sp.y > sp.x) memcpy(hb + (r * nz + sp.x) * es, comp.data() + pl.off[r] * es, (sp.y - sp.x) * es);
        }
        return FDTD_OK;
    }
    for (int64_t r = 0; r < pl.rows; ++r) {
        const int2 sp = pl.span[r];
        for (int64_t k = 0; k < nz; ++k) {
            const bool in = k >= sp.x && k < sp.y;
            const char *v = hb + (r * nz + k) * es;
            if (in) {
                memcpy(comp.data() + (pl.off[r] + k - sp.x) * es, v, es);
            } else {
                const bool nz_ = es == 8 ? *(const double *)v != 0.0 : *(const float *)v != 0.0f;
                if (nz_) return fail3(FDTD_E_INVALID, "J nonzero off the plasma support at node %lld", (long long)(r * nz + k));
            }
        }
    }
    if (pl.S > 0) HIP3(hipMemcpy(h->ws + pl.oJ[c], comp.data(), pl.S * es, hipMemcpyHostToDevice));
    return FDTD_OK;
}

int fdtd3d_get_fields(fdtd3d *h, int32_t which, void *host) { return fields_io(h, which, host, true); }

int fdtd3d_set_fields(fdtd3d *h, int32_t which, const void *host)
{
    return fields_io(h, which, const_cast<void *>(host), false);
}

int fdtd3d_steps_done(fdtd3d *h, int64_t *steps)
{
    int rc = check3(h);
    if (rc) return rc;
    if (!steps) return fail3(FDTD_E_INVALID, "steps is NULL");
    *steps = h->steps;
    return FDTD_OK;
}

int fdtd3d_profile(fdtd3d *h, int32_t on)
{
    int rc = check3(h);
    if (rc) return rc;
    HIP3(hipStreamSynchronize(h->stream));
    for (auto &r : h->recs) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    h->recs.clear();
    h->prof = on != 0;
    return FDTD_OK;
}

int fdtd3d_profile_read(fdtd3d *h, int32_t max, const char **names, double *ms, int64_t *calls, double *cells,
                        int32_t *count)
{
    int rc = check3(h);
    if (rc) return rc;
    if (!count) return fail3(FDTD_E_INVALID, "count is NULL");
    HIP3(hipStreamSynchronize(h->stream));
    double t[kKinds] = {}, c[kKinds] = {};
    int64_t n[kKinds] = {};
    for (auto &r : h->recs) {
        float e = 0.0f;
        HIP3(hipEventElapsedTime(&e, r.a, r.b));
        t[r.kind] += e;
        n[r.kind] += 1;
        c[r.kind] += r.cells;
    }
    int32_t k = 0;
    for (int i = 0; i < kKinds; ++i) {
        if (n[i] == 0) continue;
        if (k < max) {
            if (names) names[k] = kProfNames[i];
            if (ms) ms[k] = t[i];
            if (calls) calls[k] = n[i];
            if (cells) cells[k] = c[i];
        }
        ++k;
    }
    *count = k;
    return FDTD_OK;
}

int fdtd3d_destroy(fdtd3d *h)
{
    if (!h) return FDTD_OK;
    (void)hipSetDevice(h->device);
    (void)hipStreamSynchronize(h->stream);
    for (auto &kv : h->graphs) (void)hipGraphExecDestroy(kv.second);
    for (auto &r : h->recs) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    if (h->owns_ws && h->ws) (void)hipFree(h->ws);
    delete h;
    return FDTD_OK;
}

const char *fdtd3d_last_error(void) { return g_err3.c_str(); }

}  // extern "C"
