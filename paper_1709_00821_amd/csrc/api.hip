// C-ABI of the fdtd_plasma library: validation, workspace layout, host->device
// copies, time-loop orchestration (per-step, tiled, resident), graph capture,
// probe spectra.  Every step of the method runs in the HIP kernels; the host
// side only builds index tables and launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/fdtd_plasma.h"
#include "internal.h"

using namespace fdtdp;

namespace {

thread_local std::string g_last_error;

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

#define HIP_TRY(expr)                                                                   \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess)                                                           \
            return fail(FDTD_E_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

constexpr int64_t kAlign = 256;
constexpr int64_t kNodePad = 64;   // grid offsets are multiples of 64 nodes

int64_t round_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

// Workspace carve-out: a list of (offset, bytes) regions.
struct Layout {
    int64_t total = 0;
    int64_t take(int64_t bytes)
    {
        const int64_t o = total;
        total += round_up(std::max<int64_t>(bytes, 16), kAlign);
        return o;
    }
};

struct Defaults {
    int tile_cells;
    int steps_per_pass;
};

}  // namespace

// The workspace of fdtd_plasma_create_static: one file-scope device array,
// each GPU holding its own copy for the life of the process.  Host code never
// uses this name as an address (on the host it is only a stand-in for the
// symbol): the device address comes from hipGetSymbolAddress, taken once per
// device with that device current, and is kept in g_static_ws.
static __device__ __align__(256) char scratch[FDTD_STATIC_WORKSPACE_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_static_mu;
char *g_static_ws[kMaxDevices] = {};     // device address of `scratch`, per device
bool g_static_live[kMaxDevices] = {};    // a handle holds that device's copy
}  // namespace

struct fdtd_plasma {
    fdtd_plasma_desc d;
    hipStream_t stream = nullptr;
    int device = 0;
    bool owns_ws = false;
    bool static_ws = false;    // the workspace is the device's static array (create_static)
    char *ws = nullptr;
    size_t ws_bytes = 0;

    // host copies
    std::vector<int64_t> cells, off, src, probe;
    std::vector<double> freqs;
    int64_t nodes = 0;        // padded node count
    int64_t batch = 0;
    int P = 0, F = 0, SB = 0;
    int esize = 8;            // bytes per field value

    // device pointers into the workspace
    int64_t *d_off = nullptr, *d_n = nullptr, *d_src = nullptr, *d_probe = nullptr;
    double *d_wp2 = nullptr, *d_nu = nullptr, *d_freqs = nullptr, *d_samp = nullptr,
           *d_cpml = nullptr, *d_srcv = nullptr, *d_coef = nullptr;
    double2 *d_X = nullptr, *d_Xtmp = nullptr, *d_tw = nullptr;
    void *d_E[2] = {nullptr, nullptr}, *d_H[2] = {nullptr, nullptr}, *d_J[2] = {nullptr, nullptr};
    void *d_psiE[2] = {nullptr, nullptr}, *d_psiH[2] = {nullptr, nullptr};
    int64_t state_bytes = 0, psi_bytes = 0;

    // tiled executor
    std::vector<Tile> tiles_host;
    Tile *d_tiles = nullptr;
    Tile *d_adj_tiles = nullptr;   // recompute tiles of the adjoint (one list)
    int64_t n_adj_tiles = 0;
    Tile *d_rev_tiles = nullptr;   // reverse-step tiles of the adjoint (one list)
    int64_t n_rev_tiles = 0;
    double *d_adj_srcv = nullptr;  // source values of the segment being recomputed
    int64_t ntiles[kTileClasses] = {0, 0, 0, 0};
    int64_t tile_first[kTileClasses] = {0, 0, 0, 0};
    int64_t group_n[kTileClasses][kRoleGroups] = {};
    int tileC = 8, Kh = 16, tileW = 1;
    int wideC = 0;                 // class-0 tiles are 64 wideC nodes wide (0: tileC)

    // resident executor
    ResidentSlot *d_slots = nullptr;
    int64_t nbins = 0;
    int resC = 8, resWaves = 8;

    int exec = FDTD_EXEC_STEP;

    // time-loop state
    int cur = 0;
    int64_t steps = 0;        // time index of the state
    int64_t win_base = 0;     // samples of m in (win_base, win_base + SB] are buffered

    std::map<int64_t, hipGraphExec_t> graphs;
    // captured reverse sweeps, keyed by nsteps * 64 + probe: the sweep is
    // ~3 launches per step on small grids, so replaying it from a graph
    // removes most of the per-launch host cost
    std::map<int64_t, hipGraphExec_t> adj_graphs;
    bool poisoned = false;

    // side stream for the few CPML-touching tiles, which otherwise add their
    // serial latency to every pass; fork/join through events (capturable).
    // On a short grid with both CPML and role tiles, the role tiles take a
    // second side stream, so that the pass waits for the longer of the two
    // latency-bound launches instead of their sum (on a long grid the side
    // launches hide behind the bulk tiles, and the second stream's extra join
    // a pass costs more than it saves).
    hipStream_t side = nullptr, side2 = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr, ev_join2 = nullptr;

    // checkpoints (FDTD_FLAG_CHECKPOINT) and adjoint storage
    int64_t ck_T = 0;          // longest run sized for
    int64_t ck_s = 0;          // checkpoint interval
    int64_t ck_n = 0;          // checkpoint slots (steps 0, s, 2s, ...)
    bool ck_on = false;        // the advance in progress stores checkpoints
    bool ck_valid = false;     // the state is a checkpointed run() of ck_run steps
    bool tmp_valid = false;    // d_Xtmp holds the spectra of the current state (run() folds them)
    int64_t ck_run = 0;
    // recorded probe series (FDTD_FLAG_RECORD)
    int64_t rec_R = 0;         // steps kept per series row
    int64_t nfft_max = 0;
    double *d_series = nullptr;    // [batch * P][rec_R]
    double2 *d_fft[2] = {nullptr, nullptr};   // [batch * P][nfft_max] ping-pong
    char *d_ck = nullptr;      // [ck_n][3][slot_bytes]: E, H, J
    char *d_seg = nullptr;     // [ck_s + 1][3][slot_bytes]
    void *d_lam[2][3] = {{nullptr, nullptr, nullptr}, {nullptr, nullptr, nullptr}};
    double *d_grad = nullptr, *d_tab = nullptr, *d_gsrc = nullptr, *d_loss = nullptr;
    double2 *d_xref = nullptr, *d_G = nullptr;

    // per-launch timing (fdtd_plasma_profile)
    struct ProfMark {
        const char *name;
        hipEvent_t a, b;
        int64_t units;        // output nodes the launch group advances
    };
    int64_t class_nodes[kTileClasses + 1] = {0, 0, 0, 0, 0};   // output nodes per tile class; last: binned grids
    int64_t real_nodes = 0;
    bool profiling = false;
    std::vector<ProfMark> marks;

    Grids grids() const
    {
        Grids g;
        g.off = d_off;
        g.n = d_n;
        g.src = d_src;
        g.probe = d_probe;
        g.wp2 = d_wp2;
        g.nu = d_nu;
        g.coef = d_coef;
        g.coef_n = nodes;
        g.samp = d_samp;
        g.batch = batch;
        g.P = P;
        g.SB = SB;
        g.scheme = d.scheme;
        g.jdelta = d.precision == FDTD_F32_DELTA;
        g.bc = d.bc;
        g.cpmlP = d.bc == FDTD_BC_CPML ? d.cpml_cells : 0;
        g.dt = d.dt;
        g.dz = d.dz;
        g.ch = d.dt / (mu0() * d.dz);
        g.ce = d.dt / (kEps0 * d.dz);
        const double S = kC0 * d.dt / d.dz;
        g.cm = (S - 1.0) / (S + 1.0);
        g.src_tau = d.src_tau;
        g.src_t0 = d.src_t0;
        g.src_amp = d.src_amp;
        g.cpml = d_cpml;
        g.srcv = d_srcv;
        return g;
    }

    template <typename T>
    State<T> state()
    {
        State<T> s;
        for (int i = 0; i < 2; ++i) {
            s.E[i] = (T *)d_E[i];
            s.H[i] = (T *)d_H[i];
            s.J[i] = (double *)d_J[i];
            s.psiE[i] = (T *)d_psiE[i];
            s.psiH[i] = (T *)d_psiH[i];
        }
        return s;
    }
};

namespace {

int validate(const fdtd_plasma_desc *d)
{
    if (!d) return fail(FDTD_E_INVALID, "descriptor is NULL");
    if (d->struct_size != sizeof(fdtd_plasma_desc))
        return fail(FDTD_E_INVALID, "struct_size %u != %zu (header/library mismatch)",
                    d->struct_size, sizeof(fdtd_plasma_desc));
    if (d->precision != FDTD_F64 && d->precision != FDTD_F32 && d->precision != FDTD_F32_DELTA)
        return fail(FDTD_E_INVALID, "precision %d", d->precision);
    if (d->precision == FDTD_F32_DELTA &&
        ((d->exec != FDTD_EXEC_STEP && d->exec != FDTD_EXEC_TILED && d->exec != FDTD_EXEC_AUTO) ||
         (d->flags & FDTD_FLAG_CHECKPOINT) || d->tile_waves > 1 ||
         (d->tile_cells != 0 && d->tile_cells != 256 && d->tile_cells != 512)))
        return fail(FDTD_E_INVALID, "FDTD_F32_DELTA runs on the per-step executor or on one-wave register tiles "
                                    "of 256 or 512 nodes, without checkpoints");
    if (d->scheme < 0 || d->scheme > 2) return fail(FDTD_E_INVALID, "scheme %d", d->scheme);
    if (d->bc < 0 || d->bc > 2) return fail(FDTD_E_INVALID, "bc %d", d->bc);
    if (d->exec < 0 || d->exec > 4) return fail(FDTD_E_INVALID, "exec %d", d->exec);
    if (d->batch < 1) return fail(FDTD_E_INVALID, "batch %lld < 1", (long long)d->batch);
    if (!d->cells || !d->wp2 || !d->nu || !d->src_cell || !d->probe_cells || !d->freqs_hz)
        return fail(FDTD_E_INVALID, "a host array pointer is NULL");
    if (!(d->dz > 0.0) || !(d->dt > 0.0) || !std::isfinite(d->dz) || !std::isfinite(d->dt))
        return fail(FDTD_E_INVALID, "dz and dt must be positive and finite");
    if (kC0 * d->dt / d->dz > 1.0)
        return fail(FDTD_E_UNSTABLE, "Courant number c dt/dz = %.6g exceeds 1", kC0 * d->dt / d->dz);
    if (d->n_probes < 1 || d->n_freqs < 1)
        return fail(FDTD_E_INVALID, "need n_probes >= 1 and n_freqs >= 1");
    if (d->n_probes > 64) return fail(FDTD_E_INVALID, "n_probes %d > 64", d->n_probes);
    if (!(std::isfinite(d->src_tau) && d->src_tau > 0 && std::isfinite(d->src_t0) &&
          std::isfinite(d->src_amp)))
        return fail(FDTD_E_INVALID, "source parameters must be finite with tau > 0");
    for (int f = 0; f < d->n_freqs; ++f)
        if (!std::isfinite(d->freqs_hz[f])) return fail(FDTD_E_INVALID, "freqs_hz[%d] not finite", f);
    if (d->bc == FDTD_BC_CPML && d->cpml_cells < 1)
        return fail(FDTD_E_INVALID, "cpml_cells must be >= 1 with CPML ends");
    int64_t o = 0;
    for (int64_t b = 0; b < d->batch; ++b) {
        const int64_t n = d->cells[b];
        // tiles address nodes with 32-bit indices (one past the last node included)
        if (n < 3 || n > (int64_t)INT32_MAX)
            return fail(FDTD_E_INVALID, "grid %lld: cells %lld out of [3, 2^31 - 1]", (long long)b,
                        (long long)n);
        if (d->bc == FDTD_BC_CPML && 2 * (int64_t)d->cpml_cells >= n)
            return fail(FDTD_E_INVALID, "grid %lld: CPML of %d nodes per end needs more than %lld nodes",
                        (long long)b, d->cpml_cells, (long long)n);
        const int64_t s = d->src_cell[b];
        if (s != -1 && (s < 1 || s > n - 2))
            return fail(FDTD_E_INVALID, "grid %lld: source node %lld outside [1, n-2]", (long long)b,
                        (long long)s);
        for (int p = 0; p < d->n_probes; ++p) {
            const int64_t q = d->probe_cells[b * d->n_probes + p];
            if (q < 0 || q >= n)
                return fail(FDTD_E_INVALID, "grid %lld: probe %d node %lld outside [0, n)",
                            (long long)b, p, (long long)q);
        }
        for (int64_t k = 0; k < n; ++k) {
            const double w = d->wp2[o + k], v = d->nu[o + k];
            if (!(w >= 0.0) || !std::isfinite(w) || !(v >= 0.0) || !std::isfinite(v))
                return fail(FDTD_E_INVALID, "grid %lld node %lld: wp2 and nu must be finite and >= 0",
                            (long long)b, (long long)k);
            if (w != 0.0 && (k == 0 || k == n - 1))
                return fail(FDTD_E_INVALID, "grid %lld: wp2 must be 0 at the end nodes", (long long)b);
            if (w != 0.0 && d->bc == FDTD_BC_CPML &&
                (k < d->cpml_cells || k > n - 1 - d->cpml_cells))
                return fail(FDTD_E_UNSUPPORTED, "grid %lld node %lld: plasma inside the CPML layer",
                            (long long)b, (long long)k);
        }
        o += n;
    }
    if ((d->flags & FDTD_FLAG_CHECKPOINT) && (d->checkpoint_steps < 1 || d->checkpoint_steps > (1 << 30)))
        return fail(FDTD_E_INVALID, "checkpoint_steps %d out of [1, 2^30]", d->checkpoint_steps);
    if ((d->flags & FDTD_FLAG_RECORD) && (d->record_steps < 1 || d->record_steps > (1 << 24)))
        return fail(FDTD_E_INVALID, "record_steps %d out of [1, 2^24]", d->record_steps);
    if (d->flags & ~(FDTD_FLAG_CHECKPOINT | FDTD_FLAG_RECORD))
        return fail(FDTD_E_INVALID, "unknown flags 0x%x", d->flags);
    if (d->tile_cells != 0 && (d->tile_cells % 256 != 0 || d->tile_cells < 256 || d->tile_cells > 1024))
        return fail(FDTD_E_INVALID, "tile_cells %d: must be 0, 256, 512, 768 or 1024", d->tile_cells);
    if (d->tile_waves != 0 && d->tile_waves != 1 && d->tile_waves != 2 && d->tile_waves != 4 && d->tile_waves != 8)
        return fail(FDTD_E_INVALID, "tile_waves %d: must be 0, 1, 2, 4 or 8", d->tile_waves);
    if (d->tile_waves > 1 && d->tile_cells != 0 && d->tile_cells != 256 && d->tile_cells != 512)
        return fail(FDTD_E_INVALID, "tile_waves > 1 takes tile_cells 256 or 512");
    if (d->steps_per_pass != 0 && (d->steps_per_pass < 4 || d->steps_per_pass % 4 != 0 ||
                                   d->steps_per_pass > 64))
        return fail(FDTD_E_INVALID, "steps_per_pass %d: must be 0 or a multiple of 4 in [4, 64]",
                    d->steps_per_pass);
    if (d->vacuum_tile_cells != 0) {
        const int v = d->vacuum_tile_cells, t = d->tile_cells ? d->tile_cells : 512;
        if (v != 768 && v != 1024 && v != 1536 && v != 2048)
            return fail(FDTD_E_INVALID, "vacuum_tile_cells %d: must be 0, 768, 1024, 1536 or 2048", v);
        if (v <= t) return fail(FDTD_E_INVALID, "vacuum_tile_cells %d not wider than the tiles (%d)", v, t);
        if (d->tile_waves > 1 || d->precision == FDTD_F32_DELTA)
            return fail(FDTD_E_INVALID, "vacuum_tile_cells takes one-wave tiles and FDTD_F64 or FDTD_F32");
    }
    return FDTD_OK;
}

struct Plan {
    Layout L;
    int64_t o_coef = -1;      // the tiles' coefficient table (none in the FP32 ablation)
    int64_t o_off = 0, o_n = 0, o_src = 0, o_probe = 0, o_wp2 = 0, o_nu = 0, o_freqs = 0, o_samp = 0, o_srcv = 0,
            o_X = 0, o_Xtmp = 0, o_tw = 0, o_cpml = 0;
    int64_t o_E[2] = {0, 0}, o_H[2] = {0, 0}, o_J[2] = {0, 0}, o_psiE[2] = {0, 0}, o_psiH[2] = {0, 0};
    int64_t o_tiles = 0, o_slots = 0, o_adj_tiles = 0, o_adj_srcv = 0, o_rev_tiles = 0;
    std::vector<Tile> adj_tiles, rev_tiles;
    int64_t o_ck = 0, o_seg = 0, o_lam[2][3] = {{0, 0, 0}, {0, 0, 0}}, o_grad = 0, o_tab = 0,
            o_gsrc = 0, o_loss = 0, o_xref = 0, o_G = 0;
    int64_t ck_T = 0, ck_s = 0, ck_n = 0;
    int64_t rec_R = 0, nfft_max = 0, o_series = 0, o_fft[2] = {0, 0};
    int64_t nodes = 0, state_bytes = 0, psi_bytes = 0;
    int SB = 0;
    std::vector<int64_t> off;
    std::vector<Tile> tiles;
    int64_t ntiles[kTileClasses] = {0, 0, 0, 0}, tile_first[kTileClasses] = {0, 0, 0, 0};
    int64_t group_n[kTileClasses][kRoleGroups] = {};   // tiles of each role group, in group order within a class
    std::vector<ResidentSlot> slots;
    int64_t nbins = 0;
    int exec = 0, tileC = 8, Kh = 16, tileW = 1, resC = 8, resWaves = 8;
    int wideC = 0;            // wide vacuum tiles: 64 wideC nodes (0: none)
};

// Tile tables for the temporally blocked executor: per grid, outputs of width
// W = tile - 2 Kh; held span [out_lo - Kh, out_hi + Kh) clipped to the grid.
// Tiles of every grid, or of the grids skip[] does not mark.
void build_tiles(const fdtd_plasma_desc *d, Plan &p, const std::vector<char> *skip = nullptr)
{
    const int wave_nodes = p.tileC * 64;
    const int L = p.tileW * wave_nodes;
    const int W = L - 2 * p.Kh;
    const int Lw = p.wideC * 64, Ww = Lw - 2 * p.Kh;   // wide vacuum tiles (Lw = 0: none)
    std::vector<Tile> cls[kTileClasses];
    std::vector<int64_t> npl;                           // plasma nodes before node k of the grid
    int64_t o = 0;
    for (int64_t b = 0; b < d->batch; ++b) {
        const int64_t n = d->cells[b];
        const int64_t s = d->src_cell[b];
        if (Lw) {
            npl.assign(n + 1, 0);
            for (int64_t k = 0; k < n; ++k) npl[k + 1] = npl[k] + (d->wp2[o + k] != 0.0);
        }
        // a wide tile at outputs [out, out + Ww): its whole span [out - Kh,
        // out - Kh + Lw) vacuum, off both grid ends and the CPML layers, no
        // source in it and no probe among its outputs
        auto wide_ok = [&](int64_t out) {
            const int64_t lo = out - p.Kh, hi = lo + Lw;
            if (lo < 1 || hi > n - 1) return false;
            if (d->bc == FDTD_BC_CPML && (lo < d->cpml_cells + 1 || hi > n - 2 - d->cpml_cells)) return false;
            if (s >= lo && s < hi) return false;
            for (int q = 0; q < d->n_probes; ++q) {
                const int64_t pc = d->probe_cells[b * d->n_probes + q];
                if (pc >= out && pc < out + Ww) return false;
            }
            return npl[hi] == npl[lo];
        };
        for (int64_t out = 0; !(skip && (*skip)[b]) && out < n;) {
            if (Lw && wide_ok(out)) {
                Tile t{};
                t.grid = (int32_t)b;
                t.out_lo = (int32_t)out;
                t.out_hi = (int32_t)(out + Ww);
                t.lo = (int32_t)(out - p.Kh);
                t.hi = (int32_t)(out - p.Kh + Lw);
                t.flags = 0;
                cls[0].push_back(t);
                out += Ww;
                continue;
            }
            Tile t{};
            t.grid = (int32_t)b;
            t.out_lo = (int32_t)out;
            t.out_hi = (int32_t)std::min<int64_t>(n, out + W);
            t.lo = (int32_t)std::max<int64_t>(0, out - p.Kh);
            t.hi = (int32_t)std::min<int64_t>(n, (int64_t)t.lo + L);
            // a grid's last tile of a grid longer than a tile ends exactly at
            // node n (more left halo than needed, the same outputs), so node
            // n-1 always sits in the last register of the last lane
            if (t.hi == n && n >= L && p.tileW == 1) t.lo = (int32_t)(n - L);
            // node n-1 must not open a wave: its Mur update reads node n-2 by
            // an in-wave move.  Start one node earlier (node -1 reads as zero
            // and is never written); the tile still reaches n (see DESIGN).
            if (t.hi == n && n - 1 > t.lo && (n - 1 - t.lo) % wave_nodes == 0) t.lo -= 1;
            int fl = 0;
            if (t.lo <= 0) fl |= TILE_LEFT_END;
            if (t.hi == n) fl |= TILE_RIGHT_END;
            if (s >= t.lo && s < t.hi) fl |= TILE_SOURCE;
            for (int q = 0; q < d->n_probes; ++q) {
                const int64_t pc = d->probe_cells[b * d->n_probes + q];
                if (pc >= t.out_lo && pc < t.out_hi) fl |= TILE_PROBE;
            }
            for (int64_t k = std::max<int64_t>(t.lo, 0); k < t.hi; ++k)
                if (d->wp2[o + k] != 0.0) { fl |= TILE_PLASMA; break; }
            if (d->bc == FDTD_BC_CPML &&
                (t.lo < d->cpml_cells + 1 || t.hi > n - 2 - d->cpml_cells))
                fl |= TILE_CPML;
            const bool role = (fl & (TILE_LEFT_END | TILE_RIGHT_END | TILE_SOURCE | TILE_PROBE)) != 0;
            if (role && !(fl & TILE_CPML) && p.tileW == 1) {
                // the fixed-register role step applies when every role node
                // sits where it expects it
                const int C = p.tileC;
                bool fixed = true;
                if (fl & TILE_LEFT_END) fixed = fixed && t.lo == 0;
                if (fl & TILE_RIGHT_END) fixed = fixed && (int64_t)t.lo == n - L;
                if (fl & TILE_SOURCE) fixed = fixed && (s - t.lo) % C == 0;
                int np = 0;
                for (int q = 0; q < d->n_probes; ++q) {
                    const int64_t pc = d->probe_cells[b * d->n_probes + q];
                    if (pc >= t.out_lo && pc < t.out_hi) {
                        ++np;
                        fixed = fixed && (pc - t.lo) % C == 0;
                    }
                }
                if (fixed && np <= 2) fl |= TILE_FIXED;
            }
            t.flags = fl;
            // with wide vacuum tiles, class 0 holds only those; a narrow
            // vacuum tile runs with the plasma tiles (same bits)
            const int k = (fl & TILE_CPML) ? 2 : role ? 3 : ((fl & TILE_PLASMA) || Lw) ? 1 : 0;
            cls[k].push_back(t);
            out += W;
        }
        o += n;
    }
    p.tiles.clear();
    for (int k = 0; k < kTileClasses; ++k) {
        p.tile_first[k] = (int64_t)p.tiles.size();
        p.ntiles[k] = (int64_t)cls[k].size();
        for (int r = 0; r < kRoleGroups; ++r) p.group_n[k][r] = 0;
        if (k >= 2 && p.tileW == 1 && p.ntiles[k] >= kRoleGroupMinTiles) {
            // a group too small to fill the GPU would be one latency-bound
            // launch more on the side stream: its tiles join the last group,
            // launched once, each wave taking the code of its own roles
            int64_t cnt[kRoleGroups] = {};
            for (const Tile &t : cls[k]) ++cnt[role_group(t.flags)];
            auto grp = [&](const Tile &t) {
                const int r = role_group(t.flags);
                return cnt[r] < kRoleGroupMinLaunch ? kRoleGroups - 1 : r;
            };
            std::stable_sort(cls[k].begin(), cls[k].end(),
                             [&](const Tile &a, const Tile &b) { return grp(a) < grp(b); });
            for (const Tile &t : cls[k]) ++p.group_n[k][grp(t)];
        } else {
            p.group_n[k][kRoleGroups - 1] = p.ntiles[k];
        }
        p.tiles.insert(p.tiles.end(), cls[k].begin(), cls[k].end());
    }
}

// Resident bins: grids packed first-fit-decreasing into workgroups of
// resWaves waves, each grid on ceil(n / (64 C)) consecutive waves.  With
// skip_long, grids that do not fit a workgroup are left out (MIXED);
// otherwise such a grid makes the packing fail.
bool build_bins(const fdtd_plasma_desc *d, Plan &p, bool skip_long = false)
{
    const int64_t per_wave = 64LL * p.resC;
    std::vector<std::pair<int64_t, int64_t>> need;  // (waves, grid)
    std::vector<int> shift(d->batch, 0);
    for (int64_t b = 0; b < d->batch; ++b) {
        const int64_t n = d->cells[b];
        shift[b] = ((n - 1) % per_wave == 0) ? 1 : 0;
        const int64_t w = (n + shift[b] + per_wave - 1) / per_wave;
        if (w > p.resWaves) {
            if (skip_long) continue;
            return false;
        }
        need.push_back({w, b});
    }
    std::stable_sort(need.begin(), need.end(),
                     [](const std::pair<int64_t, int64_t> &a, const std::pair<int64_t, int64_t> &b) {
                         return a.first > b.first;
                     });
    std::vector<int> used;                          // waves used per bin
    std::vector<std::vector<ResidentSlot>> bins;
    for (auto &nw : need) {
        size_t j = 0;
        for (; j < bins.size(); ++j)
            if (used[j] + nw.first <= p.resWaves) break;
        if (j == bins.size()) {
            bins.emplace_back();
            used.push_back(0);
        }
        ResidentSlot s{};
        s.grid = (int32_t)nw.second;
        s.first_wave = used[j];
        s.nwaves = (int32_t)nw.first;
        s.shift = shift[nw.second];
        used[j] += (int)nw.first;
        bins[j].push_back(s);
    }
    // flatten: one entry per wave of each bin (grid -1 marks an idle wave)
    p.slots.clear();
    for (size_t j = 0; j < bins.size(); ++j) {
        std::vector<ResidentSlot> row(p.resWaves, ResidentSlot{-1, 0, 0, 0});
        for (auto &s : bins[j])
            for (int w = 0; w < s.nwaves; ++w) {
                row[s.first_wave + w] = s;
            }
        p.slots.insert(p.slots.end(), row.begin(), row.end());
    }
    p.nbins = (int64_t)bins.size();
    return true;
}

int plan(const fdtd_plasma_desc *d, Plan &p)
{
    int rc = validate(d);
    if (rc) return rc;
    const int es = d->precision == FDTD_F64 ? 8 : 4;
    const int P = d->n_probes, F = d->n_freqs;
    p.off.resize(d->batch + 1);
    int64_t o = 0;
    for (int64_t b = 0; b < d->batch; ++b) {
        p.off[b] = o;
        o += round_up(d->cells[b], kNodePad) + kNodePad;
    }
    p.off[d->batch] = o;
    p.nodes = o;
    p.state_bytes = o * es;
    p.psi_bytes = d->bc == FDTD_BC_CPML ? d->batch * 2 * d->cpml_cells * es : 16;

    // executor choice
    p.tileC = d->tile_cells ? d->tile_cells / 64 : 8;
    p.tileW = d->tile_waves ? d->tile_waves : 1;
    p.wideC = d->vacuum_tile_cells / 64;
    p.Kh = d->steps_per_pass ? d->steps_per_pass : 48;
    p.resC = 8;
    p.resWaves = 8;   // 512-thread workgroups keep the FP64 coefficients in registers without spills
    p.exec = d->exec;
    if ((p.exec == FDTD_EXEC_RESIDENT || p.exec == FDTD_EXEC_MIXED) && d->bc == FDTD_BC_CPML)
        return fail(FDTD_E_UNSUPPORTED, "the resident executor has no CPML ends");
    const int64_t res_max = resident_max_nodes(p.resC, p.resWaves);
    // AUTO takes the register tiles: on MI355X they beat the resident bins for
    // a single short grid and for batches of short grids alike (no per-step
    // barriers, no idle waves), and the bins beside tiles (MIXED) lose on the
    // 4096-slab batch; RESIDENT and MIXED stay available on request.  The
    // exception is FP32 storage on a few grids that fit the bins: there the
    // resident executor keeps the fields in FP64 registers for a whole sample
    // window, so they are rounded to FP32 once a window instead of once a
    // tile pass, which is what keeps a short run's reflection and
    // transmission at the low end of the band within the FP32 target.
    if (p.exec == FDTD_EXEC_AUTO) {
        p.exec = FDTD_EXEC_TILED;
        bool fits = d->precision == FDTD_F32 && d->bc != FDTD_BC_CPML && d->batch <= kResidentAutoGrids;
        for (int64_t b = 0; fits && b < d->batch; ++b) fits = d->cells[b] + 1 <= res_max;
        if (fits) p.exec = FDTD_EXEC_RESIDENT;
    }
    if (p.exec == FDTD_EXEC_RESIDENT) {
        if (!build_bins(d, p))
            return fail(FDTD_E_INVALID, "a grid exceeds %lld nodes, the resident limit", (long long)res_max);
    }
    if (p.exec == FDTD_EXEC_MIXED) {
        build_bins(d, p, true);
        if (p.nbins == 0) p.exec = FDTD_EXEC_TILED;      // nothing fits: plain tiles
    }
    if (p.exec == FDTD_EXEC_TILED || p.exec == FDTD_EXEC_MIXED) {
        if (p.tileW * p.tileC * 64 <= 2 * p.Kh + 64)
            return fail(FDTD_E_INVALID, "tile of %d nodes too small for halo %d", p.tileW * p.tileC * 64, p.Kh);
        // MIXED: tiles only for the grids the bins left out
        std::vector<char> binned(d->batch, 0);
        if (p.exec == FDTD_EXEC_MIXED)
            for (auto &s : p.slots)
                if (s.grid >= 0) binned[s.grid] = 1;
        build_tiles(d, p, p.exec == FDTD_EXEC_MIXED ? &binned : nullptr);
    }
    if (p.exec != FDTD_EXEC_RESIDENT && p.exec != FDTD_EXEC_MIXED) { p.slots.clear(); p.nbins = 0; }

    // sample window: up to 16384 steps, at most ~256 MiB of samples
    {
        int64_t sb = ((int64_t)1 << 28) / (8 * d->batch * P);
        sb = std::max<int64_t>(64, std::min<int64_t>(16384, sb));
        p.SB = (int)(sb / 64 * 64);
    }

    Layout &L = p.L;
    L = Layout();
    p.o_off = L.take(8 * (d->batch + 1));
    p.o_n = L.take(8 * d->batch);
    p.o_src = L.take(8 * d->batch);
    p.o_probe = L.take(8 * d->batch * P);
    p.o_freqs = L.take(8 * F);
    p.o_wp2 = L.take(8 * p.nodes);
    p.o_nu = L.take(8 * p.nodes);
    if (d->precision != FDTD_F32_DELTA) p.o_coef = L.take(8 * 4 * p.nodes);
    p.o_samp = L.take(8 * d->batch * P * (int64_t)p.SB);
    p.o_srcv = L.take(8 * (int64_t)p.SB);
    p.o_X = L.take(16 * d->batch * P * (int64_t)F);
    p.o_Xtmp = L.take(16 * d->batch * P * (int64_t)F);
    p.o_tw = L.take(16 * (int64_t)std::min(p.SB, kTwiddleChunk) * F);
    p.o_cpml = L.take(8 * 4 * std::max(1, d->cpml_cells));
    for (int i = 0; i < 2; ++i) {
        p.o_E[i] = L.take(p.state_bytes);
        p.o_H[i] = L.take(p.state_bytes);
        p.o_J[i] = L.take(8 * p.nodes);            // J in FP64 at either precision
        p.o_psiE[i] = L.take(p.psi_bytes);
        p.o_psiH[i] = L.take(p.psi_bytes);
    }
    p.o_xref = L.take(16 * d->batch * (int64_t)F);
    p.o_G = L.take(16 * d->batch * (int64_t)F);
    p.o_loss = L.take(8 * d->batch);
    if (d->flags & FDTD_FLAG_CHECKPOINT) {
        p.ck_T = d->checkpoint_steps;
        p.ck_s = (int64_t)std::ceil(std::sqrt((double)p.ck_T));
        p.ck_n = p.ck_T / p.ck_s + 1;
        const int64_t st3 = 3 * round_up(8 * p.nodes, kAlign);    // E, H, J slots sized for J
        p.o_ck = L.take(p.ck_n * st3);
        p.o_seg = L.take((p.ck_s + 1) * st3);
        for (int i = 0; i < 2; ++i)
            for (int q = 0; q < 3; ++q) p.o_lam[i][q] = L.take(p.state_bytes);
        p.o_grad = L.take(8 * p.nodes);
        p.o_tab = L.take(8 * 12 * p.nodes);
        p.o_gsrc = L.take(8 * d->batch * p.ck_T);
        // the reverse sweep recomputes each segment with register tiles of
        // kTraceCells nodes, kTraceHalo steps per launch
        Plan q;
        q.tileC = kTraceCells / 64;
        q.tileW = 1;
        q.Kh = kTraceHalo;
        build_tiles(d, q);
        p.adj_tiles = q.tiles;
        // and runs the transposed steps on tiles of kAdjCells nodes, up to
        // kAdjHalo steps per launch
        Plan r;
        r.tileC = kAdjCells / 64;
        r.tileW = 1;
        r.Kh = kAdjHalo;
        build_tiles(d, r);
        p.rev_tiles = r.tiles;
        p.o_adj_tiles = L.take((int64_t)sizeof(Tile) * std::max<size_t>(1, p.adj_tiles.size()));
        p.o_rev_tiles = L.take((int64_t)sizeof(Tile) * std::max<size_t>(1, p.rev_tiles.size()));
        p.o_adj_srcv = L.take(8 * p.ck_s);
    }
    if (d->flags & FDTD_FLAG_RECORD) {
        p.rec_R = d->record_steps;
        int64_t q = 1;
        while (q < p.rec_R + 1) q <<= 1;
        p.nfft_max = 2 * q;
        p.o_series = L.take(8 * d->batch * P * p.rec_R);
        for (int i = 0; i < 2; ++i) p.o_fft[i] = L.take(16 * d->batch * P * p.nfft_max);
    }
    p.o_tiles = L.take((int64_t)sizeof(Tile) * std::max<size_t>(1, p.tiles.size()));
    p.o_slots = L.take((int64_t)sizeof(ResidentSlot) * std::max<size_t>(1, p.slots.size()));
    return FDTD_OK;
}

template <typename T>
void zero_state(fdtd_plasma *h)
{
    for (int i = 0; i < 2; ++i) {
        launch_fill(h->d_E[i], round_up(h->state_bytes, 16), h->stream);
        launch_fill(h->d_H[i], round_up(h->state_bytes, 16), h->stream);
        launch_fill(h->d_J[i], round_up(8 * h->nodes, 16), h->stream);
        launch_fill(h->d_psiE[i], round_up(h->psi_bytes, 16), h->stream);
        launch_fill(h->d_psiH[i], round_up(h->psi_bytes, 16), h->stream);
    }
    launch_fill(h->d_X, 16 * h->batch * h->P * (int64_t)h->F, h->stream);
}

void spectra_to_tmp(fdtd_plasma *h);

void reset(fdtd_plasma *h)
{
    if (h->esize == 8) zero_state<double>(h); else zero_state<float>(h);
    h->cur = 0;
    h->steps = 0;
    h->win_base = 0;
}

// Events around one launch group while profiling (no-ops otherwise).
void prof_begin(fdtd_plasma *h, const char *name, int64_t units)
{
    if (!h->profiling) return;
    fdtd_plasma::ProfMark m{name, nullptr, nullptr, units};
    if (hipEventCreate(&m.a) != hipSuccess || hipEventCreate(&m.b) != hipSuccess) return;
    (void)hipEventRecord(m.a, h->stream);
    h->marks.push_back(m);
}

void prof_end(fdtd_plasma *h)
{
    if (!h->profiling || h->marks.empty()) return;
    (void)hipEventRecord(h->marks.back().b, h->stream);
}

// One pass of tile class c: one launch, or, for a CPML or role class sorted
// into role groups, one launch per group.
template <typename T>
void launch_class(fdtd_plasma *h, const Grids &g, State<T> &s, int cur, int c, int nsteps, int slot,
                  hipStream_t st)
{
    int64_t first = h->tile_first[c];
    // an unsplit CPML or role class (below the grouping threshold): one launch
    // whose waves each take the role code of their own group
    // (the last group of a split class is launched the same way: it holds
    // the tiles of the rarer role combinations)
    const bool one_wave = c >= 2 && h->tileW == 1;
    for (int r = 0; r < kRoleGroups; ++r) {
        const int64_t n = h->group_n[c][r];
        if (n)
            launch_tiled<T>(g, s, cur, h->d_tiles + first, n, c, c == 0 && h->wideC ? h->wideC : h->tileC,
                            nsteps, slot, st, h->tileW, one_wave && r == kRoleGroups - 1 ? -1 : r);
        first += n;
    }
}

// Copy the samples of the current window (full or partial) into the
// recorded series.
void record_window(fdtd_plasma *h)
{
    if (h->d_series)
        launch_series_copy(h->d_samp, h->SB, h->batch * h->P, (int)(h->steps - h->win_base), h->d_series,
                           h->rec_R, h->win_base, h->stream);
}

// Fold the full sample window into X (and into the recorded series).
void flush(fdtd_plasma *h)
{
    record_window(h);
    const int count = (int)(h->steps - h->win_base);
    prof_begin(h, "dft_flush", 0);
    launch_dft(h->grids(), h->d_freqs, h->F, h->win_base + 1, count, h->d_tw, h->d_X,
               h->batch * h->P, h->stream);
    prof_end(h);
    h->win_base = h->steps;
}

template <typename T>
int advance_t(fdtd_plasma *h, int64_t nsteps)
{
    const Grids g = h->grids();
    State<T> s = h->state<T>();
    int64_t left = nsteps;
    const int64_t ck3 = 3 * round_up(8 * h->nodes, kAlign);
    while (left > 0) {
        const int slot = (int)(h->steps - h->win_base);
        int64_t room = h->SB - slot;
        // a new sample window: source values of all its steps, read by the
        // register-tile kernels
        if (slot == 0) {
            prof_begin(h, "source_table", 0);
            launch_src_table(g, h->steps + 1, h->SB, h->d_srcv, h->stream);
            prof_end(h);
        }
        if (h->ck_on) {
            if (h->steps % h->ck_s == 0 && h->steps / h->ck_s < h->ck_n) {
                char *dst = h->d_ck + (h->steps / h->ck_s) * ck3;
                const int64_t sb = round_up(8 * h->nodes, kAlign);
                launch_copy(dst, h->d_E[h->cur], round_up(h->state_bytes, 16), h->stream);
                launch_copy(dst + sb, h->d_H[h->cur], round_up(h->state_bytes, 16), h->stream);
                launch_copy(dst + 2 * sb, h->d_J[h->cur], round_up(8 * h->nodes, 16), h->stream);
            }
            room = std::min<int64_t>(room, h->ck_s - h->steps % h->ck_s);
        }
        int64_t k;
        static const char *kTiledNames[kTileClasses] = {"tiled_vacuum", "tiled_plasma", "tiled_cpml",
                                                        "tiled_role"};
        if (h->exec == FDTD_EXEC_STEP) {
            k = 1;
            prof_begin(h, "step_h_e", h->real_nodes);
            launch_step<T>(g, s, h->cur, h->nodes, h->steps + 1, slot, h->stream);
            prof_end(h);
        } else if (h->exec == FDTD_EXEC_TILED) {
            k = std::min<int64_t>(std::min<int64_t>(left, room), h->Kh);
            // the CPML and role classes (the tiles holding grid ends, sources
            // and probes) run beside the bulk classes on the side stream: all
            // classes of a pass write disjoint nodes
            const bool fork = h->side && (h->ntiles[2] || h->ntiles[3]) && !h->profiling;
            auto on_side = [&](int c) { return fork && c >= 2; };
            if (fork) {
                (void)hipEventRecord(h->ev_fork, h->stream);
                (void)hipStreamWaitEvent(h->side, h->ev_fork, 0);
                if (h->side2) {
                    (void)hipStreamWaitEvent(h->side2, h->ev_fork, 0);
                    launch_class<T>(h, g, s, h->cur, 2, (int)k, slot, h->side);
                    launch_class<T>(h, g, s, h->cur, 3, (int)k, slot, h->side2);
                    (void)hipEventRecord(h->ev_join2, h->side2);
                } else {
                    for (int c = 2; c < kTileClasses; ++c)
                        launch_class<T>(h, g, s, h->cur, c, (int)k, slot, h->side);
                }
                (void)hipEventRecord(h->ev_join, h->side);
            }
            for (int c = 0; c < kTileClasses; ++c)
                if (h->ntiles[c] && !on_side(c)) {
                    prof_begin(h, kTiledNames[c], h->class_nodes[c]);
                    launch_class<T>(h, g, s, h->cur, c, (int)k, slot, h->stream);
                    prof_end(h);
                }
            if (fork) {
                (void)hipStreamWaitEvent(h->stream, h->ev_join, 0);
                if (h->side2) (void)hipStreamWaitEvent(h->stream, h->ev_join2, 0);
            }
        } else if (h->exec == FDTD_EXEC_MIXED) {
            // bins and tiles hold disjoint grids.  The bins advance the whole
            // window in one launch (beside the tiles on the side stream, unless
            // profiling) and write the buffer the tile passes end in.
            k = std::min<int64_t>(left, room);
            const int64_t passes = (k + h->Kh - 1) / h->Kh;
            const int out = h->cur ^ (int)(passes & 1);
            const bool fork = h->side && !h->profiling;
            hipStream_t rs = fork ? h->side : h->stream;
            if (fork) {
                (void)hipEventRecord(h->ev_fork, h->stream);
                (void)hipStreamWaitEvent(h->side, h->ev_fork, 0);
            }
            prof_begin(h, "resident", h->class_nodes[kTileClasses]);
            launch_resident<T>(g, s, h->cur, out, h->d_slots, h->nbins, h->resWaves, h->resC, (int)k, slot,
                               rs);
            prof_end(h);
            if (fork) (void)hipEventRecord(h->ev_join, h->side);
            int cur = h->cur;
            for (int64_t done = 0; done < k; done += h->Kh) {
                const int kk = (int)std::min<int64_t>(h->Kh, k - done);
                for (int c = 0; c < kTileClasses; ++c)
                    if (h->ntiles[c]) {
                        prof_begin(h, kTiledNames[c], h->class_nodes[c]);
                        launch_class<T>(h, g, s, cur, c, kk, slot + (int)done, h->stream);
                        prof_end(h);
                    }
                cur ^= 1;
            }
            if (fork) (void)hipStreamWaitEvent(h->stream, h->ev_join, 0);
            h->cur = out ^ 1;          // flipped back below
        } else {
            k = std::min<int64_t>(left, room);
            prof_begin(h, "resident", h->real_nodes);
            launch_resident<T>(g, s, h->cur, h->cur, h->d_slots, h->nbins, h->resWaves, h->resC, (int)k, slot,
                               h->stream);
            prof_end(h);
        }
        if (h->exec != FDTD_EXEC_RESIDENT) h->cur ^= 1;
        h->steps += k;
        left -= k;
        if (h->steps - h->win_base == h->SB) flush(h);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(FDTD_E_DEVICE, "kernel launch failed: %s", hipGetErrorString(e));
    return FDTD_OK;
}

int advance(fdtd_plasma *h, int64_t nsteps)
{
    return h->esize == 8 ? advance_t<double>(h, nsteps) : advance_t<float>(h, nsteps);
}

int check_handle(fdtd_plasma *h)
{
    if (!h) return fail(FDTD_E_INVALID, "handle is NULL");
    if (h->poisoned) return fail(FDTD_E_STATE, "handle used after a device failure");
    return FDTD_OK;
}

}  // namespace

extern "C" {

const char *fdtd_plasma_last_error(void) { return g_last_error.c_str(); }

int fdtd_plasma_workspace_bytes(const fdtd_plasma_desc *desc, size_t *bytes)
{
    if (!bytes) return fail(FDTD_E_INVALID, "bytes is NULL");
    Plan p;
    int rc = plan(desc, p);
    if (rc) return rc;
    *bytes = (size_t)p.L.total;
    return FDTD_OK;
}

}  // extern "C"

namespace {

// create with a planned descriptor; static_ws: the workspace is the device's
// static array (no side stream or events are made, so the handle allocates
// nothing but its host object)
int create_impl(const fdtd_plasma_desc *desc, Plan &p, void *dev_workspace, size_t workspace_bytes,
                fdtd_plasma **out, bool static_ws);

}  // namespace

extern "C" {

int fdtd_plasma_create(const fdtd_plasma_desc *desc, void *dev_workspace, size_t workspace_bytes,
                       fdtd_plasma **out)
{
    if (!out) return fail(FDTD_E_INVALID, "out is NULL");
    *out = nullptr;
    Plan p;
    int rc = plan(desc, p);
    if (rc) return rc;
    return create_impl(desc, p, dev_workspace, workspace_bytes, out, false);
}

int fdtd_plasma_create_static(const fdtd_plasma_desc *desc, fdtd_plasma **out)
{
    if (!out) return fail(FDTD_E_INVALID, "out is NULL");
    *out = nullptr;
    Plan p;
    int rc = plan(desc, p);
    if (rc) return rc;
    if (p.L.total > (int64_t)FDTD_STATIC_WORKSPACE_BYTES)
        return fail(FDTD_E_WORKSPACE, "the descriptor needs a %lld-byte workspace, above the %lld-byte static one",
                    (long long)p.L.total, (long long)FDTD_STATIC_WORKSPACE_BYTES);
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(FDTD_E_DEVICE, "device %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_static_mu);
    if (g_static_live[dev])
        return fail(FDTD_E_STATE, "a handle on device %d already holds the static workspace", dev);
    if (!g_static_ws[dev]) {
        void *ptr = nullptr;
        HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        g_static_ws[dev] = (char *)ptr;
    }
    rc = create_impl(desc, p, g_static_ws[dev], (size_t)FDTD_STATIC_WORKSPACE_BYTES, out, true);
    if (rc == FDTD_OK) g_static_live[dev] = true;
    return rc;
}

}  // extern "C"

namespace {

int create_impl(const fdtd_plasma_desc *desc, Plan &p, void *dev_workspace, size_t workspace_bytes,
                fdtd_plasma **out, bool static_ws)
{
    int rc = FDTD_OK;
    if (dev_workspace && workspace_bytes < (size_t)p.L.total)
        return fail(FDTD_E_WORKSPACE, "workspace of %zu bytes < %lld needed", workspace_bytes,
                    (long long)p.L.total);
    if (dev_workspace && ((uintptr_t)dev_workspace % kAlign))
        return fail(FDTD_E_WORKSPACE, "workspace not %lld-byte aligned", (long long)kAlign);

    fdtd_plasma *h = new (std::nothrow) fdtd_plasma();
    if (!h) return fail(FDTD_E_INVALID, "out of host memory");
    h->static_ws = static_ws;
    h->d = *desc;
    h->stream = (hipStream_t)desc->stream;
    h->batch = desc->batch;
    h->P = desc->n_probes;
    h->F = desc->n_freqs;
    h->SB = p.SB;
    h->esize = desc->precision == FDTD_F64 ? 8 : 4;
    h->nodes = p.nodes;
    h->state_bytes = p.state_bytes;
    h->psi_bytes = p.psi_bytes;
    h->exec = p.exec;
    h->tileC = p.tileC;
    h->wideC = p.wideC;
    h->tileW = p.tileW;
    h->Kh = p.Kh;
    h->resC = p.resC;
    h->resWaves = p.resWaves;
    h->nbins = p.nbins;
    for (int k = 0; k < kTileClasses; ++k) {
        h->ntiles[k] = p.ntiles[k];
        h->tile_first[k] = p.tile_first[k];
        for (int r = 0; r < kRoleGroups; ++r) h->group_n[k][r] = p.group_n[k][r];
        for (int64_t t = 0; t < p.ntiles[k]; ++t) {
            const Tile &tl = p.tiles[p.tile_first[k] + t];
            h->class_nodes[k] += tl.out_hi - tl.out_lo;
        }
    }
    for (int64_t b = 0; b < desc->batch; ++b) h->real_nodes += desc->cells[b];
    {
        std::vector<char> binned(desc->batch, 0);
        for (auto &sl : p.slots)
            if (sl.grid >= 0) binned[sl.grid] = 1;
        for (int64_t b = 0; b < desc->batch; ++b)
            if (binned[b]) h->class_nodes[kTileClasses] += desc->cells[b];
    }
    h->cells.assign(desc->cells, desc->cells + desc->batch);
    h->off = p.off;
    h->src.assign(desc->src_cell, desc->src_cell + desc->batch);
    h->probe.assign(desc->probe_cells, desc->probe_cells + desc->batch * desc->n_probes);
    h->freqs.assign(desc->freqs_hz, desc->freqs_hz + desc->n_freqs);
    h->d.cells = nullptr;
    h->d.wp2 = h->d.nu = nullptr;
    h->d.src_cell = h->d.probe_cells = nullptr;
    h->d.freqs_hz = nullptr;

    auto undo = [&](int code) {
        if (h->side) (void)hipStreamDestroy(h->side);
        if (h->side2) (void)hipStreamDestroy(h->side2);
        if (h->ev_fork) (void)hipEventDestroy(h->ev_fork);
        if (h->ev_join) (void)hipEventDestroy(h->ev_join);
        if (h->ev_join2) (void)hipEventDestroy(h->ev_join2);
        if (h->owns_ws && h->ws) (void)hipFree(h->ws);
        delete h;
        return code;
    };
    if (hipGetDevice(&h->device) != hipSuccess) return undo(fail(FDTD_E_DEVICE, "no HIP device"));
    if (dev_workspace) {
        h->ws = (char *)dev_workspace;
        h->ws_bytes = workspace_bytes;
    } else {
        hipError_t e = hipMalloc((void **)&h->ws, (size_t)p.L.total);
        if (e != hipSuccess)
            return undo(fail(FDTD_E_DEVICE, "hipMalloc(%lld) failed: %s", (long long)p.L.total,
                             hipGetErrorString(e)));
        h->owns_ws = true;
        h->ws_bytes = (size_t)p.L.total;
    }
    char *w = h->ws;
    h->d_off = (int64_t *)(w + p.o_off);
    h->d_n = (int64_t *)(w + p.o_n);
    h->d_src = (int64_t *)(w + p.o_src);
    h->d_probe = (int64_t *)(w + p.o_probe);
    h->d_freqs = (double *)(w + p.o_freqs);
    h->d_wp2 = (double *)(w + p.o_wp2);
    h->d_nu = (double *)(w + p.o_nu);
    h->d_coef = p.o_coef >= 0 ? (double *)(w + p.o_coef) : nullptr;
    h->d_samp = (double *)(w + p.o_samp);
    h->d_srcv = (double *)(w + p.o_srcv);
    h->d_X = (double2 *)(w + p.o_X);
    h->d_Xtmp = (double2 *)(w + p.o_Xtmp);
    h->d_tw = (double2 *)(w + p.o_tw);
    h->d_cpml = (double *)(w + p.o_cpml);
    for (int i = 0; i < 2; ++i) {
        h->d_E[i] = w + p.o_E[i];
        h->d_H[i] = w + p.o_H[i];
        h->d_J[i] = w + p.o_J[i];
        h->d_psiE[i] = w + p.o_psiE[i];
        h->d_psiH[i] = w + p.o_psiH[i];
    }
    h->d_xref = (double2 *)(w + p.o_xref);
    h->d_G = (double2 *)(w + p.o_G);
    h->d_loss = (double *)(w + p.o_loss);
    h->ck_T = p.ck_T;
    h->ck_s = p.ck_s;
    h->ck_n = p.ck_n;
    if (desc->flags & FDTD_FLAG_CHECKPOINT) {
        h->d_ck = w + p.o_ck;
        h->d_seg = w + p.o_seg;
        for (int i = 0; i < 2; ++i)
            for (int q = 0; q < 3; ++q) h->d_lam[i][q] = w + p.o_lam[i][q];
        h->d_grad = (double *)(w + p.o_grad);
        h->d_tab = (double *)(w + p.o_tab);
        h->d_gsrc = (double *)(w + p.o_gsrc);
    }
    if (desc->flags & FDTD_FLAG_RECORD) {
        h->rec_R = p.rec_R;
        h->nfft_max = p.nfft_max;
        h->d_series = (double *)(w + p.o_series);
        for (int i = 0; i < 2; ++i) h->d_fft[i] = (double2 *)(w + p.o_fft[i]);
    }
    h->d_tiles = (Tile *)(w + p.o_tiles);
    if (p.o_adj_tiles) {
        h->d_adj_tiles = (Tile *)(w + p.o_adj_tiles);
        h->n_adj_tiles = (int64_t)p.adj_tiles.size();
        h->d_adj_srcv = (double *)(w + p.o_adj_srcv);
        h->d_rev_tiles = (Tile *)(w + p.o_rev_tiles);
        h->n_rev_tiles = (int64_t)p.rev_tiles.size();
    }
    h->d_slots = (ResidentSlot *)(w + p.o_slots);

    // padded material arrays (zero in the padding)
    std::vector<double> wp2(p.nodes, 0.0), nu(p.nodes, 0.0);
    {
        int64_t o = 0;
        for (int64_t b = 0; b < desc->batch; ++b) {
            std::memcpy(&wp2[p.off[b]], desc->wp2 + o, 8 * desc->cells[b]);
            std::memcpy(&nu[p.off[b]], desc->nu + o, 8 * desc->cells[b]);
            o += desc->cells[b];
        }
    }
    hipStream_t st = h->stream;
    auto H2D = [&](void *dst, const void *src, size_t bytes) {
        return hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st);
    };
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = H2D(h->d_off, p.off.data(), 8 * (desc->batch + 1));
    if (e == hipSuccess) e = H2D(h->d_n, desc->cells, 8 * desc->batch);
    if (e == hipSuccess) e = H2D(h->d_src, desc->src_cell, 8 * desc->batch);
    if (e == hipSuccess) e = H2D(h->d_probe, desc->probe_cells, 8 * desc->batch * desc->n_probes);
    if (e == hipSuccess) e = H2D(h->d_freqs, desc->freqs_hz, 8 * desc->n_freqs);
    if (e == hipSuccess) e = H2D(h->d_wp2, wp2.data(), 8 * p.nodes);
    if (e == hipSuccess) e = H2D(h->d_nu, nu.data(), 8 * p.nodes);
    if (e == hipSuccess && !p.tiles.empty())
        e = H2D(h->d_tiles, p.tiles.data(), sizeof(Tile) * p.tiles.size());
    if (e == hipSuccess && !p.slots.empty())
        e = H2D(h->d_slots, p.slots.data(), sizeof(ResidentSlot) * p.slots.size());
    if (e == hipSuccess && !p.adj_tiles.empty())
        e = H2D(h->d_adj_tiles, p.adj_tiles.data(), sizeof(Tile) * p.adj_tiles.size());
    if (e == hipSuccess && !p.rev_tiles.empty())
        e = H2D(h->d_rev_tiles, p.rev_tiles.data(), sizeof(Tile) * p.rev_tiles.size());
    if (e != hipSuccess)
        return undo(fail(FDTD_E_DEVICE, "host-to-device copy failed: %s", hipGetErrorString(e)));
    if (h->d_coef) launch_coef1d(h->grids(), p.nodes, h->d_coef, st);
    if (desc->bc == FDTD_BC_CPML) {
        const double m = desc->cpml_m > 0 ? desc->cpml_m : 3.0;
        const double eta0 = std::sqrt(mu0() / kEps0);
        const double smax = desc->cpml_sigma_max > 0 ? desc->cpml_sigma_max
                                                     : 0.8 * (m + 1.0) / (eta0 * desc->dz);
        launch_cpml_table(h->d_cpml, desc->cpml_cells, m, smax, desc->dt, st);
    }
    if (((h->exec == FDTD_EXEC_TILED && (h->ntiles[2] > 0 || h->ntiles[3] > 0)) || h->exec == FDTD_EXEC_MIXED) &&
        h->stream != nullptr && !static_ws) {
        // default priority (no priority streams), non-blocking w.r.t. the null stream
        if (hipStreamCreateWithFlags(&h->side, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&h->ev_fork, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&h->ev_join, hipEventDisableTiming) != hipSuccess)
            return undo(fail(FDTD_E_DEVICE, "side stream creation failed"));
        if (h->exec == FDTD_EXEC_TILED && h->ntiles[2] > 0 && h->ntiles[3] > 0 &&
            h->ntiles[0] + h->ntiles[1] < kSide2MaxBulkTiles &&
            (hipStreamCreateWithFlags(&h->side2, hipStreamNonBlocking) != hipSuccess ||
             hipEventCreateWithFlags(&h->ev_join2, hipEventDisableTiming) != hipSuccess))
            return undo(fail(FDTD_E_DEVICE, "side stream creation failed"));
    }
    reset(h);
    // the host staging vectors die with this scope: wait for the copies
    e = hipStreamSynchronize(st);
    if (e == hipSuccess) e = hipGetLastError();
    if (e != hipSuccess) return undo(fail(FDTD_E_DEVICE, "create failed: %s", hipGetErrorString(e)));
    *out = h;
    return rc;
}

}  // namespace

extern "C" {

int fdtd_plasma_step(fdtd_plasma *h, int64_t nsteps)
{
    int rc = check_handle(h);
    if (rc) return rc;
    if (nsteps < 0) return fail(FDTD_E_INVALID, "nsteps %lld < 0", (long long)nsteps);
    if (nsteps > 0) h->ck_valid = false;
    h->tmp_valid = false;
    return advance(h, nsteps);
}

int fdtd_plasma_run(fdtd_plasma *h, int64_t nsteps)
{
    int rc = check_handle(h);
    if (rc) return rc;
    if (nsteps < 0) return fail(FDTD_E_INVALID, "nsteps %lld < 0", (long long)nsteps);
    h->ck_on = h->d_ck != nullptr && nsteps <= h->ck_T;
    h->ck_valid = false;
    h->tmp_valid = false;
    if (h->stream == nullptr) {
        // the legacy null stream cannot be captured: run eagerly
        reset(h);
        rc = advance(h, nsteps);
        if (rc == FDTD_OK && nsteps > 0) {
            spectra_to_tmp(h);
            h->tmp_valid = true;
        }
        h->ck_valid = h->ck_on && rc == FDTD_OK;
        h->ck_run = nsteps;
        h->ck_on = false;
        return rc;
    }
    const int64_t key = nsteps * 2 + (h->ck_on ? 1 : 0);
    auto it = h->graphs.find(key);
    if (it == h->graphs.end()) {
        // capture reset + the whole time loop once for this length
        HIP_TRY(hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
        reset(h);
        rc = advance(h, nsteps);
        // the run's last, partially filled sample window is folded into the
        // spectra inside the run (into d_Xtmp, so the running sums of d_X stay
        // as a later step() continuing the window expects them)
        if (rc == FDTD_OK && nsteps > 0) spectra_to_tmp(h);
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamEndCapture(h->stream, &graph);
        if (rc) { h->ck_on = false; if (graph) (void)hipGraphDestroy(graph); return rc; }
        if (e != hipSuccess) return fail(FDTD_E_DEVICE, "graph capture failed: %s", hipGetErrorString(e));
        hipGraphExec_t exec = nullptr;
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) return fail(FDTD_E_DEVICE, "graph instantiate failed: %s", hipGetErrorString(e));
        it = h->graphs.emplace(key, exec).first;
    } else {
        // bookkeeping identical to what the captured launches did
        h->cur = 0;
        h->steps = 0;
        h->win_base = 0;
        int64_t left = nsteps;
        while (left > 0) {
            const int slot = (int)(h->steps - h->win_base);
            int64_t room = h->SB - slot;
            if (h->ck_on) room = std::min<int64_t>(room, h->ck_s - h->steps % h->ck_s);
            int64_t k = h->exec == FDTD_EXEC_STEP ? 1
                        : h->exec == FDTD_EXEC_TILED ? std::min<int64_t>(std::min<int64_t>(left, room), h->Kh)
                                                     : std::min<int64_t>(left, room);
            if (h->exec == FDTD_EXEC_MIXED) h->cur ^= (int)(((k + h->Kh - 1) / h->Kh) & 1);
            else if (h->exec != FDTD_EXEC_RESIDENT) h->cur ^= 1;
            h->steps += k;
            left -= k;
            if (h->steps - h->win_base == h->SB) h->win_base = h->steps;
        }
    }
    HIP_TRY(hipGraphLaunch(it->second, h->stream));
    h->tmp_valid = nsteps > 0;
    h->ck_valid = h->ck_on;
    h->ck_run = nsteps;
    h->ck_on = false;
    return FDTD_OK;
}

int fdtd_plasma_steps_done(fdtd_plasma *h, int64_t *steps)
{
    int rc = check_handle(h);
    if (rc) return rc;
    if (!steps) return fail(FDTD_E_INVALID, "steps is NULL");
    *steps = h->steps;
    return FDTD_OK;
}

int fdtd_plasma_probe_spectra(fdtd_plasma *h, double *re, double *im)
{
    int rc = check_handle(h);
    if (rc) return rc;
    if (!re || !im) return fail(FDTD_E_INVALID, "output pointer is NULL");
    if (h->steps == 0) return fail(FDTD_E_STATE, "no step taken yet");
    const int64_t rows = h->batch * h->P, nX = rows * h->F;
    // X plus the partial window, without disturbing the running sums (run()
    // has folded it already)
    if (!h->tmp_valid) spectra_to_tmp(h);
    std::vector<double2> X(nX);
    HIP_TRY(hipMemcpyAsync(X.data(), h->d_Xtmp, 16 * nX, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    bool finite = true;
    for (int64_t i = 0; i < nX; ++i) {
        re[i] = X[i].x;
        im[i] = X[i].y;
        finite = finite && std::isfinite(X[i].x) && std::isfinite(X[i].y);
    }
    if (!finite) return fail(FDTD_E_NONFINITE, "a probe spectrum holds NaN or Inf");
    return FDTD_OK;
}

int fdtd_plasma_probe_series(fdtd_plasma *h, double *out)
{
    int rc = check_handle(h);
    if (rc) return rc;
    if (!out) return fail(FDTD_E_INVALID, "output pointer is NULL");
    if (!h->d_series) return fail(FDTD_E_STATE, "created without FDTD_FLAG_RECORD");
    if (h->steps < 1 || h->steps > h->rec_R)
        return fail(FDTD_E_STATE, "%lld steps done, the series holds 1 .. %lld", (long long)h->steps,
                    (long long)h->rec_R);
    const int64_t rows = h->batch * h->P;
    record_window(h);   // the partially filled window (its samples stay buffered)
    std::vector<double> buf(rows * h->rec_R);
    HIP_TRY(hipMemcpyAsync(buf.data(), h->d_series, 8 * rows * h->rec_R, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    for (int64_t r = 0; r < rows; ++r)
        std::memcpy(out + r * h->steps, buf.data() + r * h->rec_R, 8 * h->steps);
    return FDTD_OK;
}

int fdtd_plasma_probe_fft(fdtd_plasma *h, int64_t nfft, double *re, double *im)
{
    int rc = check_handle(h);
    if (rc) return rc;
    if (!re || !im) return fail(FDTD_E_INVALID, "output pointer is NULL");
    if (!h->d_series) return fail(FDTD_E_STATE, "created without FDTD_FLAG_RECORD");
    if (h->steps < 1 || h->steps > h->rec_R)
        return fail(FDTD_E_STATE, "%lld steps done, the series holds 1 .. %lld", (long long)h->steps,
                    (long long)h->rec_R);
    if (nfft <= h->steps || nfft > h->nfft_max || (nfft & (nfft - 1)) != 0)
        return fail(FDTD_E_INVALID, "nfft %lld: a power of 2 in (%lld, %lld]", (long long)nfft,
                    (long long)h->steps, (long long)h->nfft_max);
    const int64_t rows = h->batch * h->P;
    record_window(h);
    double2 *res = launch_fft(h->d_series, h->rec_R, rows, h->steps, nfft, h->d.dt, h->d_fft[0], h->d_fft[1],
                              h->stream);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(FDTD_E_DEVICE, "FFT launch failed: %s", hipGetErrorString(e));
    std::vector<double2> X(rows * nfft);
    HIP_TRY(hipMemcpyAsync(X.data(), res, 16 * rows * nfft, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    for (int64_t i = 0; i < rows * nfft; ++i) {
        re[i] = X[i].x;
        im[i] = X[i].y;
    }
    return FDTD_OK;
}

int fdtd_plasma_get_fields(fdtd_plasma *h, int64_t grid, double *E, double *H, double *J)
{
    int rc = check_handle(h);
    if (rc) return rc;
    if (grid < 0 || grid >= h->batch) return fail(FDTD_E_INVALID, "grid %lld out of range", (long long)grid);
    const int64_t n = h->cells[grid], o = h->off[grid];
    std::vector<char> buf(n * 8);
    auto fetch = [&](void *base, double *dst, int64_t cnt, int es) -> int {
        if (!dst) return FDTD_OK;
        HIP_TRY(hipMemcpyAsync(buf.data(), (char *)base + o * es, cnt * es, hipMemcpyDeviceToHost,
                               h->stream));
        HIP_TRY(hipStreamSynchronize(h->stream));
        for (int64_t k = 0; k < cnt; ++k)
            dst[k] = es == 8 ? ((double *)buf.data())[k] : (double)((float *)buf.data())[k];
        return FDTD_OK;
    };
    if ((rc = fetch(h->d_E[h->cur], E, n, h->esize))) return rc;
    if ((rc = fetch(h->d_H[h->cur], H, n - 1, h->esize))) return rc;
    if ((rc = fetch(h->d_J[h->cur], J, n, 8))) return rc;
    if (J && h->d.precision != FDTD_F32_DELTA) {
        // the state carries Q^{n-1} = CJ (J^n - b2 E^n): J^n = Q / CJ + b2 E^n,
        // with CJ and b2 of eqs.(11)+(13) from the node's wp2 and nu
        std::vector<double> En(n), w(n), v(n);
        if ((rc = fetch(h->d_E[h->cur], En.data(), n, h->esize))) return rc;
        if ((rc = fetch(h->d_wp2, w.data(), n, 8))) return rc;
        if ((rc = fetch(h->d_nu, v.data(), n, 8))) return rc;
        for (int64_t k = 0; k < n; ++k)
            if (w[k] != 0.0) {
                const Coef c = node_coef(w[k], v[k], h->d.dt, h->d.dz, h->d.scheme);
                J[k] = std::fma(c.b2, En[k], J[k] / c.CJ);
            }
    }
    return FDTD_OK;
}

}  // extern "C"

namespace {

// Spectra including the partially filled sample window, into h->d_Xtmp.
void spectra_to_tmp(fdtd_plasma *h)
{
    const int64_t rows = h->batch * h->P, nX = rows * h->F;
    launch_copy(h->d_Xtmp, h->d_X, 16 * nX, h->stream);   // a kernel: capturable
    const int count = (int)(h->steps - h->win_base);
    launch_dft(h->grids(), h->d_freqs, h->F, h->win_base + 1, count, h->d_tw, h->d_Xtmp, rows,
               h->stream);
}

int upload_xref(fdtd_plasma *h, const double *xr, const double *xi)
{
    const int64_t nx = h->batch * h->F;
    std::vector<double2> x(nx);
    for (int64_t i = 0; i < nx; ++i) {
        if (!std::isfinite(xr[i]) || !std::isfinite(xi[i]) || (xr[i] == 0.0 && xi[i] == 0.0))
            return fail(FDTD_E_INVALID, "xref[%lld] must be finite and nonzero", (long long)i);
        x[i] = make_double2(xr[i], xi[i]);
    }
    HIP_TRY(hipMemcpyAsync(h->d_xref, x.data(), 16 * nx, hipMemcpyHostToDevice, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    return FDTD_OK;
}

// Reverse sweep: per segment, recompute the forward states from its
// checkpoint into the segment buffer, then transpose the steps in reverse.
template <typename T>
int reverse_sweep(fdtd_plasma *h, int64_t Tn, int probe)
{
    Grids g = h->grids();
    Grids gt = g;                      // recompute: no probe samples, the segment's source table
    gt.P = 0;
    gt.srcv = h->d_adj_srcv;
    gt.SB = (int)h->ck_s;
    const int64_t sb = round_up(8 * h->nodes, kAlign), ck3 = 3 * sb;
    auto segE = [&](int64_t i) { return (T *)(h->d_seg + i * ck3); };
    auto segH = [&](int64_t i) { return (T *)(h->d_seg + i * ck3 + sb); };
    auto segJ = [&](int64_t i) { return (double *)(h->d_seg + i * ck3 + 2 * sb); };
    for (int i = 0; i < 2; ++i)
        for (int q = 0; q < 3; ++q) launch_fill(h->d_lam[i][q], round_up(h->state_bytes, 16), h->stream);
    launch_fill(h->d_grad, round_up(8 * h->nodes, 16), h->stream);
    int lc = 0;                        // lambda^{m+1} lives in d_lam[lc]
    const int64_t nseg = (Tn + h->ck_s - 1) / h->ck_s;
    for (int64_t j = nseg - 1; j >= 0; --j) {
        const int64_t m0 = j * h->ck_s, m1 = std::min<int64_t>(Tn, m0 + h->ck_s);
        launch_copy(h->d_seg, h->d_ck + j * ck3, ck3, h->stream);
        // forward states of steps m0 .. m1 into the segment slots 0 .. m1 - m0,
        // kTraceHalo steps per launch
        launch_src_table(g, m0 + 1, (int)(m1 - m0), h->d_adj_srcv, h->stream);
        for (int64_t i = 0; i < m1 - m0; i += kTraceHalo)
            launch_trace<T>(gt, h->d_seg, ck3, sb, h->d_adj_tiles, h->n_adj_tiles,
                            (int)std::min<int64_t>(kTraceHalo, m1 - m0 - i), (int)i, h->stream);
        if (h->exec == FDTD_EXEC_STEP) {
            // the per-step reference: one launch per transposed step
            for (int64_t m = m1 - 1; m >= m0; --m) {
                const int64_t i = m - m0;
                const T *lam[3] = {(const T *)h->d_lam[lc][0], (const T *)h->d_lam[lc][1],
                                   (const T *)h->d_lam[lc][2]};
                T *out[3] = {(T *)h->d_lam[lc ^ 1][0], (T *)h->d_lam[lc ^ 1][1], (T *)h->d_lam[lc ^ 1][2]};
                launch_adj_step<T>(g, lam, out, segE(i), segJ(i), segH(i + 1), segE(i + 1), h->d_tab,
                                   h->nodes, h->d_gsrc, Tn, m, probe, h->d_grad, h->stream);
                lc ^= 1;
            }
        } else {
            // register tiles: up to kAdjHalo transposed steps per launch, same bits
            for (int64_t mt = m1 - 1; mt >= m0; mt -= kAdjHalo) {
                const int k = (int)std::min<int64_t>(kAdjHalo, mt - m0 + 1);
                AdjTileArgs<T> a;
                a.lE = (const T *)h->d_lam[lc][0];
                a.lH = (const T *)h->d_lam[lc][1];
                a.lJ = (const T *)h->d_lam[lc][2];
                a.nE = (T *)h->d_lam[lc ^ 1][0];
                a.nH = (T *)h->d_lam[lc ^ 1][1];
                a.nJ = (T *)h->d_lam[lc ^ 1][2];
                a.tab = h->d_tab;
                a.total = h->nodes;
                a.seg = h->d_seg;
                a.slot_bytes = ck3;
                a.arr_bytes = sb;
                a.m0 = m0;
                a.gsrc = h->d_gsrc;
                a.T_ = Tn;
                a.probe = probe;
                a.grad = h->d_grad;
                launch_adj_tiled<T>(g, a, h->d_rev_tiles, h->n_rev_tiles, mt, k, h->stream);
                lc ^= 1;
            }
        }
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(FDTD_E_DEVICE, "adjoint launch failed: %s", hipGetErrorString(e));
    return FDTD_OK;
}

}  // namespace

extern "C" {

int fdtd_plasma_loss_r2(fdtd_plasma *h, int32_t probe, const double *xref_re, const double *xref_im,
                        double *loss)
{
    int rc = check_handle(h);
    if (rc) return rc;
    if (!xref_re || !xref_im || !loss) return fail(FDTD_E_INVALID, "output/input pointer is NULL");
    if (probe < 0 || probe >= h->P) return fail(FDTD_E_INVALID, "probe %d out of range", probe);
    if (h->steps == 0) return fail(FDTD_E_STATE, "no step taken yet");
    if ((rc = upload_xref(h, xref_re, xref_im))) return rc;
    spectra_to_tmp(h);
    launch_adj_prepare(h->d_Xtmp, h->batch, h->P, h->F, probe, h->d_xref, h->d_G, h->d_loss, h->stream);
    HIP_TRY(hipMemcpyAsync(loss, h->d_loss, 8 * h->batch, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    return FDTD_OK;
}

int fdtd_plasma_grad_r2(fdtd_plasma *h, int64_t nsteps, int32_t probe, const double *xref_re,
                        const double *xref_im, double *loss, double *grad)
{
    int rc = check_handle(h);
    if (rc) return rc;
    if (!xref_re || !xref_im || !loss || !grad) return fail(FDTD_E_INVALID, "a pointer is NULL");
    if (!h->d_ck) return fail(FDTD_E_STATE, "created without FDTD_FLAG_CHECKPOINT");
    if (nsteps < 1 || nsteps > h->ck_T)
        return fail(FDTD_E_INVALID, "nsteps %lld outside [1, checkpoint_steps=%lld]",
                    (long long)nsteps, (long long)h->ck_T);
    if (probe < 0 || probe >= h->P) return fail(FDTD_E_INVALID, "probe %d out of range", probe);
    if (h->d.scheme != FDTD_SCHEME_CONSISTENT || (h->d.bc != FDTD_BC_MUR1 && h->d.bc != FDTD_BC_PEC))
        return fail(FDTD_E_UNSUPPORTED, "the adjoint needs the consistent scheme and Mur or PEC ends");
    if ((rc = upload_xref(h, xref_re, xref_im))) return rc;
    if (!(h->ck_valid && h->ck_run == nsteps && h->steps == nsteps)) {
        if ((rc = fdtd_plasma_run(h, nsteps))) return rc;
    }
    spectra_to_tmp(h);
    launch_adj_prepare(h->d_Xtmp, h->batch, h->P, h->F, probe, h->d_xref, h->d_G, h->d_loss, h->stream);
    launch_adj_source(h->d_freqs, h->F, h->d.dt, h->d_G, h->batch, nsteps, h->d_gsrc, h->stream);
    launch_adj_coef(h->grids(), h->nodes, h->d_tab, h->stream);
    if (h->stream == nullptr) {
        // the legacy null stream cannot be captured: launch eagerly
        rc = h->esize == 8 ? reverse_sweep<double>(h, nsteps, probe) : reverse_sweep<float>(h, nsteps, probe);
        if (rc) return rc;
    } else {
        const int64_t key = nsteps * 64 + probe;
        auto it = h->adj_graphs.find(key);
        if (it == h->adj_graphs.end()) {
            HIP_TRY(hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
            rc = h->esize == 8 ? reverse_sweep<double>(h, nsteps, probe) : reverse_sweep<float>(h, nsteps, probe);
            hipGraph_t graph = nullptr;
            hipError_t e = hipStreamEndCapture(h->stream, &graph);
            if (rc || e != hipSuccess) {
                if (graph) (void)hipGraphDestroy(graph);
                return rc ? rc : fail(FDTD_E_DEVICE, "adjoint graph capture failed: %s", hipGetErrorString(e));
            }
            hipGraphExec_t exec = nullptr;
            e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (e != hipSuccess) return fail(FDTD_E_DEVICE, "adjoint graph instantiate failed: %s", hipGetErrorString(e));
            it = h->adj_graphs.emplace(key, exec).first;
        }
        HIP_TRY(hipGraphLaunch(it->second, h->stream));
    }
    // the sweep works in the segment buffer: fields, spectra and checkpoints
    // still hold the forward run, so another loss can reuse it
    std::vector<double> gpad(h->nodes);
    HIP_TRY(hipMemcpyAsync(gpad.data(), h->d_grad, 8 * h->nodes, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipMemcpyAsync(loss, h->d_loss, 8 * h->batch, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    int64_t o = 0;
    for (int64_t b = 0; b < h->batch; ++b) {
        std::memcpy(grad + o, gpad.data() + h->off[b], 8 * h->cells[b]);
        o += h->cells[b];
    }
    return FDTD_OK;
}

int fdtd_plasma_profile(fdtd_plasma *h, int64_t nsteps, int32_t max, char *names, double *ms_total,
                        int64_t *calls, int64_t *units, int32_t *count)
{
    int rc = check_handle(h);
    if (rc) return rc;
    if (nsteps < 0 || max < 1 || !names || !ms_total || !calls || !units || !count)
        return fail(FDTD_E_INVALID, "profile: bad arguments");
    h->profiling = true;
    h->marks.clear();
    rc = advance(h, nsteps);
    h->profiling = false;
    hipError_t e = hipStreamSynchronize(h->stream);
    std::vector<std::string> nm;
    std::vector<double> ms;
    std::vector<int64_t> cnt, un;
    for (auto &m : h->marks) {
        float t = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&t, m.a, m.b);
        size_t j = 0;
        for (; j < nm.size(); ++j)
            if (nm[j] == m.name) break;
        if (j == nm.size()) { nm.push_back(m.name); ms.push_back(0.0); cnt.push_back(0); un.push_back(0); }
        ms[j] += t;
        cnt[j] += 1;
        un[j] += m.units;
        (void)hipEventDestroy(m.a);
        (void)hipEventDestroy(m.b);
    }
    h->marks.clear();
    if (rc) return rc;
    if (e != hipSuccess) return fail(FDTD_E_DEVICE, "profile: %s", hipGetErrorString(e));
    const int nout = (int)std::min<size_t>(nm.size(), (size_t)max);
    for (int j = 0; j < nout; ++j) {
        std::memset(names + 32 * j, 0, 32);
        std::strncpy(names + 32 * j, nm[j].c_str(), 31);
        ms_total[j] = ms[j];
        calls[j] = cnt[j];
        units[j] = un[j];
    }
    *count = nout;
    return FDTD_OK;
}

int fdtd_plasma_destroy(fdtd_plasma *h)
{
    if (!h) return FDTD_OK;
    (void)hipStreamSynchronize(h->stream);
    if (h->side) {
        (void)hipStreamSynchronize(h->side);
        (void)hipStreamDestroy(h->side);
    }
    if (h->side2) {
        (void)hipStreamSynchronize(h->side2);
        (void)hipStreamDestroy(h->side2);
    }
    if (h->ev_fork) (void)hipEventDestroy(h->ev_fork);
    if (h->ev_join) (void)hipEventDestroy(h->ev_join);
    if (h->ev_join2) (void)hipEventDestroy(h->ev_join2);
    for (auto &kv : h->graphs) (void)hipGraphExecDestroy(kv.second);
    for (auto &kv : h->adj_graphs) (void)hipGraphExecDestroy(kv.second);
    if (h->owns_ws && h->ws) (void)hipFree(h->ws);
    if (h->static_ws) {
        std::lock_guard<std::mutex> lock(g_static_mu);
        g_static_live[h->device] = false;
    }
    delete h;
    return FDTD_OK;
}

}  // extern "C"
