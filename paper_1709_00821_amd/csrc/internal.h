// Internal interfaces between the host library (api.hip) and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "physics.h"

namespace fdtdp {

// Device view of all grids of a handle (passed by value to kernels).
struct Grids {
    const int64_t *off;     // [batch] first node of grid b in the padded node arrays
    const int64_t *n;       // [batch] nodes of grid b
    const int64_t *src;     // [batch] source node or -1
    const int64_t *probe;   // [batch * P] probe nodes
    const double *wp2;      // [nodes] plasma frequency^2
    const double *nu;       // [nodes] collision frequency
    const double *coef;     // [4][nodes] the register tiles' step coefficients of every node
                            // (node_coef_t<double>: eP, -CH, a, qc), built once; null in
                            // the FP32 ablation, whose tiles build their own
    int64_t coef_n;         // row length of coef (the padded node count)
    double *samp;           // [batch * P][SB] probe samples of the current window
    int64_t batch;
    int P;                  // probes per grid
    int SB;                 // sample window length
    int scheme;
    int jdelta;             // FP32 ablation: eq.(11) in FP32 with FP32 delta-form coefficients
    int bc;                 // FDTD_BC_*
    int cpmlP;              // CPML nodes per end (bc = CPML)
    double dt, dz;
    double ch;              // dt/(mu0 dz)
    double ce;              // dt/(eps0 dz)
    double cm;              // Mur coefficient (S-1)/(S+1)
    double src_tau, src_t0, src_amp;
    const double *cpml;     // [4][cpmlP]: bE(depth d+1), aE(d+1), bH(depth j+1/2), aH(j+1/2)
    const double *srcv;     // [SB] eq.(15) source value of every step of the current window
};

// State buffers of one precision.
template <typename T>
struct State {
    T *E[2];
    T *H[2];
    double *J[2];           // the plasma current, in FP64 at either field precision, carried as
                            // Q^{n-1} = CJ (J^n - b2 E^n) (the FP32 ablation: J^n itself)
    T *psiE[2];             // [batch][2][P]: left zone then right zone
    T *psiH[2];
};

struct Launch {
    hipStream_t stream;
};

// One tile of the temporally blocked kernel (node indices local to the grid).
struct Tile {
    int32_t grid;
    int32_t lo;        // first node held
    int32_t hi;        // one past the last node held (<= n)
    int32_t out_lo;    // first node written back
    int32_t out_hi;    // one past the last node written back
    int32_t flags;     // TILE_* bits
    int32_t pad0, pad1;
};

enum {
    TILE_LEFT_END = 1,    // node 0 held
    TILE_RIGHT_END = 2,   // node n-1 held
    TILE_SOURCE = 4,      // the grid's source node held
    TILE_PROBE = 8,       // a probe node among the written-back nodes
    TILE_PLASMA = 16,     // some held node has wp2 > 0
    TILE_CPML = 32,       // some held node lies in a CPML layer
    TILE_FIXED = 64       // a one-wave role tile whose role nodes sit where the fixed-register
                          // role step expects them: node 0 at register 0 of lane 0, node n-1 at
                          // register C-1 of lane 63, the source and at most two probes at
                          // register 0 of their lanes
};

// One workgroup of the resident kernel: waves [w0, w1) of a bin hold grid g's
// nodes [node0, node0 + waves*64*C).
struct ResidentSlot {
    int32_t grid;
    int32_t first_wave;   // wave index (within the workgroup) holding node 0
    int32_t nwaves;       // waves used by this grid
    int32_t shift;        // 1: node k sits at position k+1 (keeps n-2, n-1 in one lane)
};

// AUTO picks the resident executor for FP32 storage on at most this many grids
// when all of them fit the bins (see plan() in api.hip).
constexpr int64_t kResidentAutoGrids = 16;
// Samples folded into the DFT per twiddle table (table: kTwiddleChunk x F).
constexpr int kTwiddleChunk = 1024;
// Tile classes of the temporally blocked executor: 0 vacuum, 1 plasma (both
// without grid ends, source or probes), 2 tiles touching a CPML layer, 3 the
// other tiles holding a grid end, the source or a probe.
constexpr int kTileClasses = 4;
// The CPML and role classes take a stream each (instead of sharing one) only
// while the bulk classes hold fewer tiles than one round of the plasma
// kernel on the GPU (three waves a SIMD): then every launch of a pass is
// latency bound.  Measured: the 1000-step paper setup at 10,240 cells 0.88 ->
// 0.60 ms with two streams; the 2^24-node grid 82.6 -> 90.7 ms.
constexpr int64_t kSide2MaxBulkTiles = 3072;

// Roles a one-wave tile may hold, as bits of a mask.  A CPML or role class
// with at least kRoleGroupMinTiles tiles is sorted into role groups and each
// group is launched with the role step compiled for its mask (a tile holding
// only the right end then runs no source or left-end code); smaller classes,
// whose launches are latency bound, take one launch with the full step.  The
// probe part, and the source part, still check at run time whether the tile
// has one.
// kRoleFixed: the role nodes sit at the registers TILE_FIXED names, so the
// role step addresses them directly instead of picking registers at run time.
enum : int { kRoleSrc = 1, kRoleLeft = 2, kRoleRight = 4, kRoleProbe = 8, kRoleAll = 15, kRoleFixed = 16 };
constexpr int kRoleGroups = 11;
constexpr int64_t kRoleGroupMinTiles = 2048;
constexpr int64_t kRoleGroupMinLaunch = 1024;   // smaller groups join the last one
// group of a tile from its TILE_* flags: probe only, source, left end, right
// end, left end and source (0-4), the same five with TILE_FIXED (5-9),
// anything else (10)
inline int role_group(int flags)
{
    const int m = ((flags & TILE_SOURCE) ? kRoleSrc : 0) | ((flags & TILE_LEFT_END) ? kRoleLeft : 0) |
                  ((flags & TILE_RIGHT_END) ? kRoleRight : 0);
    int r;
    switch (m) {
    case 0: r = 0; break;
    case kRoleSrc: r = 1; break;
    case kRoleLeft: r = 2; break;
    case kRoleRight: r = 3; break;
    case kRoleLeft | kRoleSrc: r = 4; break;
    default: return kRoleGroups - 1;
    }
    return (flags & TILE_FIXED) ? r + 5 : r;
}

// ---- kernel launchers (kernels1d.hip) ------------------------------------
template <typename T>
void launch_step(const Grids &g, State<T> &s, int cur, int64_t total_nodes, int64_t m,
                 int slot, hipStream_t st);

// Tiles of `waves` waves (1: one wave a tile, neighbours by DPP only; 2, 4,
// 8: one workgroup a tile, neighbouring waves through LDS).
// group: the role group of every tile of a CPML or role-class launch of
// one-wave tiles (kRoleGroups - 1: the full role step; -1: a small mixed
// class, each wave picking the code of its own group).
template <typename T>
void launch_tiled(const Grids &g, State<T> &s, int cur, const Tile *tiles, int64_t ntiles,
                  int klass, int C, int nsteps, int slot0, hipStream_t st, int waves = 1,
                  int group = kRoleGroups - 1);

// Forward recompute of nsteps steps from segment slot slot0, every step's
// state stored (tiles of kTraceCells nodes with a kTraceHalo halo, nsteps <=
// kTraceHalo).
template <typename T>
void launch_trace(const Grids &g, char *seg, int64_t slot_bytes, int64_t arr_bytes, const Tile *tiles,
                  int64_t ntiles, int nsteps, int slot0, hipStream_t st);
constexpr int kTraceCells = 128, kTraceHalo = 48;

// Reverse sweep on register tiles (kAdjCells nodes, kAdjHalo halo): nsteps
// transposed steps m = mtop, mtop - 1, .. per launch.
template <typename T>
struct AdjTileArgs {
    const T *lE, *lH, *lJ;      // lambda^{mtop+1} (read)
    T *nE, *nH, *nJ;            // lambda^{mtop+1-nsteps} (written, output nodes)
    const double *tab;          // [12][total] coefficients, wp2-derivatives and 1/CJ
    int64_t total;
    const char *seg;            // forward states: slot i = m - m0 (E, H at + arr_bytes, the carried
                                // Q = CJ (J - b2 E) at + 2 arr_bytes)
    int64_t slot_bytes, arr_bytes, m0;
    const double *gsrc;         // [batch][T_] dL/dE at the probe
    int64_t T_;
    int probe;
    double *grad;               // [total]
};
template <typename T>
void launch_adj_tiled(const Grids &g, const AdjTileArgs<T> &a, const Tile *tiles, int64_t ntiles, int64_t mtop,
                      int nsteps, hipStream_t st);
constexpr int kAdjCells = 128, kAdjHalo = 48;
constexpr int kAdjPrefetch = 6;   // steps of forward state the reverse sweep loads ahead

// Reads buffer cur, writes buffer out (cur itself for a whole-run resident
// call, the other buffer when bins and tiles share a pass).
template <typename T>
void launch_resident(const Grids &g, State<T> &s, int cur, int out, const ResidentSlot *slots,
                     int64_t nbins, int waves_per_wg, int C, int nsteps, int slot0, hipStream_t st);

void launch_dft(const Grids &g, const double *freqs, int F, int64_t m_first, int count,
                double2 *tw, double2 *X, int64_t rows, hipStream_t st);

void launch_fill(void *p, int64_t bytes, hipStream_t st);

// ---- recorded series and FFT (fft1d.hip) ----------------------------------
// series[row][m0 + i] = samp[row][i] (i < count, m0 + i < R)
void launch_series_copy(const double *samp, int SB, int64_t rows, int count, double *series, int64_t R,
                        int64_t m0, hipStream_t st);
// dt-scaled zero-padded FFT (nfft points) of the first `steps` entries of every
// series row (entry m-1 at time m); returns the one of buf0, buf1 holding it
double2 *launch_fft(const double *series, int64_t R, int64_t rows, int64_t steps, int64_t nfft, double dt,
                    double2 *buf0, double2 *buf1, hipStream_t st);
// srcv[i] = source value of step m_first + i, i < count (eq.(15) at t = m dt)
void launch_src_table(const Grids &g, int64_t m_first, int count, double *srcv, hipStream_t st);

void launch_cpml_table(double *tab, int P, double m, double smax, double dt, hipStream_t st);

int resident_max_nodes(int C, int waves);

// ---- adjoint (adjoint1d.hip) -----------------------------------------------
// The register tiles' coefficient table from wp2 and nu (once per create).
void launch_coef1d(const Grids &g, int64_t total, double *coef, hipStream_t st);
void launch_adj_coef(const Grids &g, int64_t total, double *tab, hipStream_t st);
void launch_adj_prepare(const double2 *X, int64_t batch, int P, int F, int probe,
                        const double2 *xref, double2 *G, double *loss, hipStream_t st);
void launch_adj_source(const double *freqs, int F, double dt, const double2 *G, int64_t batch,
                       int64_t T, double *gsrc, hipStream_t st);
template <typename T>
void launch_adj_step(const Grids &g, const T *const lam[3], T *const out[3], const T *En,
                     const double *Jn, const T *Hh, const T *En1, const double *tab, int64_t total,
                     const double *gsrc, int64_t T_, int64_t m, int probe, double *grad,
                     hipStream_t st);
void launch_copy(void *dst, const void *src, int64_t bytes, hipStream_t st);

}  // namespace fdtdp
