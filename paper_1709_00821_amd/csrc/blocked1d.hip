// Register-resident 1D kernels for gfx950.
//
// Each lane holds C consecutive nodes of E, H (and J, coefficients in plasma,
// psi in CPML layers) in VGPRs; a wave holds 64*C consecutive nodes.  One
// time step needs two neighbour values per lane: E of the next lane's first
// node (for its last H) and H of the previous lane's last node (for its first
// E), moved with cross-lane shuffles; all other neighbours are in the lane.
//
//  * k_tiled: temporal blocking.  Every wave is an independent tile holding
//    its output nodes plus Kh halo nodes on each side; it runs K <= Kh steps
//    with no synchronisation at all (the invalid region grows one node per
//    step from each cut edge and never reaches the outputs), then writes the
//    output nodes to the other ping-pong buffer.
//  * k_resident: one workgroup keeps whole grids (packed into its waves) in
//    registers for the entire call; waves of one grid swap edge values
//    through LDS with two barriers per step.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace fdtdp {

// ------------------------------------------------------------ chunk state

template <typename T, int C, bool PLASMA, bool CPML>
struct Chunk {
    T E[C], H[C];
    double J[PLASMA ? C : 1];      // the current, held in FP64
    double Ed[PLASMA ? C : 1];     // E^n widened to FP64 (the J update's E_old), kept across steps
    NodeCoef<T> cf[PLASMA ? C : 1];
    uint32_t pmask;                // bit i: node i is plasma
    T pE[CPML ? C : 1], pH[CPML ? C : 1];
    T bE[CPML ? C : 1], aE[CPML ? C : 1], bH[CPML ? C : 1], aH[CPML ? C : 1];
    uint32_t eZone, hZone;         // bit i: node i has an E / H psi
};

template <typename T>
struct BitsOf;
template <>
struct BitsOf<float> {
    using type = uint32_t;
};
template <>
struct BitsOf<double> {
    using type = uint64_t;
};

// Value of v[i] for a runtime i in [0, C) (0 bits if none matches).  Written
// as an OR of masked bit patterns: a chain of value selects would be folded
// into one load through a selected address, which forces the register array
// into scratch memory.
template <typename T, int C>
__device__ __forceinline__ T pick(const T (&v)[C], int i)
{
    using U = typename BitsOf<T>::type;
    U r = 0;
#pragma unroll
    for (int j = 0; j < C; ++j) r |= (i == j) ? __builtin_bit_cast(U, v[j]) : (U)0;
    return __builtin_bit_cast(T, r);
}

// a if c else b, without a select between two loads (see pick)
template <typename T>
__device__ __forceinline__ T choose(bool c, T a, T b)
{
    using U = typename BitsOf<T>::type;
    const U m = c ? ~(U)0 : (U)0;
    return __builtin_bit_cast(T, (U)((__builtin_bit_cast(U, a) & m) | (__builtin_bit_cast(U, b) & ~m)));
}

template <typename T, int C>
__device__ __forceinline__ void put(T (&v)[C], int i, T x)
{
#pragma unroll
    for (int j = 0; j < C; ++j)
        if (i == j) v[j] = x;
}

// Whole-wave neighbour moves with DPP (gfx9 wave_shl:1 / wave_shr:1): lane i
// receives lane i+1's value (down) or lane i-1's (up); the lane with no source
// receives 0.  One v_mov_b32_dpp per 32-bit half, no LDS crossbar trip.
__device__ __forceinline__ int dpp_down1(int x)
{
    return __builtin_amdgcn_update_dpp(0, x, 0x130, 0xF, 0xF, false);
}
__device__ __forceinline__ int dpp_up1(int x)
{
    return __builtin_amdgcn_update_dpp(0, x, 0x138, 0xF, 0xF, false);
}
__device__ __forceinline__ float shfl_down1(float x)
{
    return __builtin_bit_cast(float, dpp_down1(__builtin_bit_cast(int, x)));
}
__device__ __forceinline__ float shfl_up1(float x)
{
    return __builtin_bit_cast(float, dpp_up1(__builtin_bit_cast(int, x)));
}
__device__ __forceinline__ double shfl_down1(double x)
{
    const int2 v = __builtin_bit_cast(int2, x);
    return __builtin_bit_cast(double, make_int2(dpp_down1(v.x), dpp_down1(v.y)));
}
__device__ __forceinline__ double shfl_up1(double x)
{
    const int2 v = __builtin_bit_cast(int2, x);
    return __builtin_bit_cast(double, make_int2(dpp_up1(v.x), dpp_up1(v.y)));
}

// Load nodes [k0, k0+C) of array a (grid-local pointer); nodes >= lim read 0.
template <typename T, int C>
__device__ __forceinline__ void load_chunk(const T *a, int64_t k0, int64_t lim, T (&v)[C])
{
    constexpr int per16 = 16 / (int)sizeof(T);
    if (k0 >= 0 && k0 + C <= lim && (k0 % per16) == 0) {
        constexpr int per = per16;
        static_assert(C % per == 0, "C must fill 16-byte vectors");
        const uint4 *p = reinterpret_cast<const uint4 *>(a + k0);
#pragma unroll
        for (int q = 0; q < C / per; ++q) {
            const uint4 u = p[q];
            const T *t = reinterpret_cast<const T *>(&u);
#pragma unroll
            for (int r = 0; r < per; ++r) v[q * per + r] = t[r];
        }
    } else {
#pragma unroll
        for (int i = 0; i < C; ++i) v[i] = (k0 + i < lim && k0 + i >= 0) ? a[k0 + i] : (T)0;
    }
}

// Store nodes [k0, k0+C) restricted to [lo, hi).
template <typename T, int C>
__device__ __forceinline__ void store_chunk(T *a, int64_t k0, int64_t lo, int64_t hi, const T (&v)[C])
{
    constexpr int per16 = 16 / (int)sizeof(T);
    if (k0 >= lo && k0 + C <= hi && (k0 % per16) == 0) {
        constexpr int per = per16;
        uint4 *p = reinterpret_cast<uint4 *>(a + k0);
#pragma unroll
        for (int q = 0; q < C / per; ++q) {
            uint4 u;
            T *t = reinterpret_cast<T *>(&u);
#pragma unroll
            for (int r = 0; r < per; ++r) t[r] = v[q * per + r];
            p[q] = u;
        }
    } else {
#pragma unroll
        for (int i = 0; i < C; ++i)
            if (k0 + i >= lo && k0 + i < hi) a[k0 + i] = v[i];
    }
}

// Load the lane's chunk starting at grid node k0 of grid b (buffer `buf`).
template <typename T, int C, bool PLASMA, bool CPML>
__device__ __forceinline__ void chunk_load(Chunk<T, C, PLASMA, CPML> &ck, const Grids &g,
                                           const State<T> &s, int buf, int b, int64_t off,
                                           int64_t n, int64_t k0, int64_t lim)
{
    load_chunk<T, C>(s.E[buf] + off, k0, lim, ck.E);
    load_chunk<T, C>(s.H[buf] + off, k0, lim, ck.H);
    ck.pmask = 0;
    if constexpr (PLASMA) {
        load_chunk<double, C>(s.J[buf] + off, k0, lim, ck.J);
#pragma unroll
        for (int i = 0; i < C; ++i) ck.Ed[i] = (double)ck.E[i];
        double w[C], v[C];
        load_chunk<double, C>(g.wp2 + off, k0, lim, w);
        load_chunk<double, C>(g.nu + off, k0, lim, v);
#pragma unroll
        for (int i = 0; i < C; ++i) {
            if (w[i] != 0.0) ck.pmask |= 1u << i;
            ck.cf[i] = node_coef_t<T>(w[i], v[i], g.dt, g.dz, g.scheme);
        }
    }
    if constexpr (CPML) {
        ck.eZone = ck.hZone = 0;
        const int P = g.cpmlP;
#pragma unroll
        for (int i = 0; i < C; ++i) {
            const int64_t k = k0 + i;
            ck.pE[i] = ck.pH[i] = (T)0;
            ck.bE[i] = ck.bH[i] = (T)1;
            ck.aE[i] = ck.aH[i] = (T)0;
            if (k < 0 || k >= lim) continue;   // k = -1: a tile shifted off node 0
            int slot = -1, tab = 0;
            // E psi: nodes 1..P-1 and n-P..n-2 (depth d -> table d-1)
            if (k >= 1 && k < P) { tab = P - 1 - (int)k; slot = (int)k; }
            else if (k > n - 1 - P && k <= n - 2) { tab = (int)(k - (n - 1 - P)) - 1; slot = P + (int)(k - (n - P)); }
            if (slot >= 0) {
                ck.eZone |= 1u << i;
                ck.pE[i] = s.psiE[buf][(int64_t)b * 2 * P + slot];
                ck.bE[i] = (T)g.cpml[tab];
                ck.aE[i] = (T)g.cpml[P + tab];
            }
            slot = -1;
            // H psi: nodes 0..P-1 and n-1-P..n-2 (depth j+1/2 -> table j)
            if (k < P) { tab = P - 1 - (int)k; slot = (int)k; }
            else if (k >= n - 1 - P && k <= n - 2) { tab = (int)(k - (n - 1 - P)); slot = P + tab; }
            if (slot >= 0) {
                ck.hZone |= 1u << i;
                ck.pH[i] = s.psiH[buf][(int64_t)b * 2 * P + slot];
                ck.bH[i] = (T)g.cpml[2 * P + tab];
                ck.aH[i] = (T)g.cpml[3 * P + tab];
            }
        }
    }
}

template <typename T, int C, bool PLASMA, bool CPML>
__device__ __forceinline__ void chunk_store(const Chunk<T, C, PLASMA, CPML> &ck, const Grids &g,
                                            const State<T> &s, int buf, int b, int64_t off,
                                            int64_t n, int64_t k0, int64_t lo, int64_t hi)
{
    store_chunk<T, C>(s.E[buf] + off, k0, lo, hi, ck.E);
    store_chunk<T, C>(s.H[buf] + off, k0, lo, hi < n ? hi : n - 1, ck.H);   // H has n-1 nodes
    if constexpr (PLASMA) store_chunk<double, C>(s.J[buf] + off, k0, lo, hi, ck.J);
    if constexpr (CPML) {
        const int P = g.cpmlP;
#pragma unroll
        for (int i = 0; i < C; ++i) {
            const int64_t k = k0 + i;
            if (k < lo || k >= hi) continue;
            if (ck.eZone & (1u << i)) {
                const int slot = (k < P) ? (int)k : P + (int)(k - (n - P));
                s.psiE[buf][(int64_t)b * 2 * P + slot] = ck.pE[i];
            }
            if (ck.hZone & (1u << i)) {
                const int slot = (k < P) ? (int)k : P + (int)(k - (n - 1 - P));
                s.psiH[buf][(int64_t)b * 2 * P + slot] = ck.pH[i];
            }
        }
    }
}

// H^{n+1/2} of the chunk; Er = E of the next node after the chunk.
template <typename T, int C, bool PLASMA, bool CPML>
__device__ __forceinline__ void chunk_h(Chunk<T, C, PLASMA, CPML> &ck, T Er, T ch)
{
#pragma unroll
    for (int i = 0; i < C; ++i) {
        const T er = (i + 1 < C) ? ck.E[i + 1] : Er;
        if constexpr (CPML) {
            if (ck.hZone & (1u << i)) {
                const T dE = er - ck.E[i];
                ck.pH[i] = fmat(ck.aH[i], dE, ck.bH[i] * ck.pH[i]);
                ck.H[i] = fmat(-ch, dE + ck.pH[i], ck.H[i]);
                continue;
            }
        }
        ck.H[i] = h_update<T>(ck.H[i], ck.E[i], er, ch);
    }
}

// E^{n+1} (before the source) of the chunk; Hl = H of the node before the
// chunk.
template <typename T, int C, bool PLASMA, bool CPML>
__device__ __forceinline__ void chunk_e(Chunk<T, C, PLASMA, CPML> &ck, T Hl, T ce)
{
#pragma unroll
    for (int i = 0; i < C; ++i) {
        T curl = ck.H[i] - ((i > 0) ? ck.H[i - 1] : Hl);
        if constexpr (CPML) {
            if (ck.eZone & (1u << i)) {
                ck.pE[i] = fmat(ck.aE[i], curl, ck.bE[i] * ck.pE[i]);
                curl = curl + ck.pE[i];
            }
        }
        if constexpr (PLASMA) {
            // the plasma formula reproduces the vacuum update at vacuum nodes
            ck.E[i] = e_update_plasma(ck.E[i], ck.J[i], curl, ck.cf[i]);
        } else {
            ck.E[i] = e_update_vac<T>(ck.E[i], curl, ce);
        }
    }
}

// J update of the chunk (after the source), with E_old the FP64 copy of E^n
// kept from the previous step; at vacuum nodes a*0 + 0*E + 0*E keeps J at +0.
// The Mur ends rewrite E after this and leave their copy stale, which is
// harmless: end nodes carry no plasma (b1 = 0).
template <typename T, int C, bool PLASMA, bool CPML>
__device__ __forceinline__ void chunk_j(Chunk<T, C, PLASMA, CPML> &ck)
{
    if constexpr (PLASMA) {
#pragma unroll
        for (int i = 0; i < C; ++i) {
            const double en = (double)ck.E[i];
            ck.J[i] = j_update<T>(ck.J[i], ck.Ed[i], en, ck.cf[i]);
            ck.Ed[i] = en;
        }
    }
}

// One time step of a chunk that holds no grid end and no source: H, E, J only.
template <typename T, int C, bool PLASMA, bool CPML, typename GetEr, typename GetHl>
__device__ __forceinline__ void chunk_step_plain(Chunk<T, C, PLASMA, CPML> &ck, const Grids &g,
                                                 GetEr get_er, GetHl get_hl)
{
    chunk_h<T, C, PLASMA, CPML>(ck, get_er(ck.E[0]), (T)g.ch);
    chunk_e<T, C, PLASMA, CPML>(ck, get_hl(ck.H[C - 1]), (T)g.ce);
    chunk_j<T, C, PLASMA, CPML>(ck);
}

// Everything a lane needs to know about the grid ends, source and probes in
// its chunk (computed once per launch).
struct ChunkRole {
    int isrc;        // index of the source node in the chunk, or -1
    int ileft;       // index of node 0 in the chunk (0 or 1; node 1 follows it), or -1
    int iright;      // index of node n-1 in the chunk, or -1
    bool right_any;  // some lane of the wave holds node n-1
    bool left_any;
    bool src_any;
};

// One full time step of a lane's chunk.  Er / Hl come from the neighbours;
// the caller supplies them through get_er() / get_hl() so both kernels share
// this body.
template <typename T, int C, bool PLASMA, bool CPML, typename GetEr, typename GetHl>
__device__ __forceinline__ void chunk_step(Chunk<T, C, PLASMA, CPML> &ck, const Grids &g,
                                           const ChunkRole &role, int64_t m, GetEr get_er,
                                           GetHl get_hl)
{
    const T ch = (T)g.ch, ce = (T)g.ce;
    // E^n values the Mur ends need
    const int il = role.ileft > 0 ? 1 : 0;
    T eo0 = choose<T>(il, ck.E[1], ck.E[0]), eo1 = choose<T>(il, ck.E[2], ck.E[1]);
    T eoR = (T)0, eoR1 = (T)0;
    if (role.right_any) {
        const T prevLast = shfl_up1(ck.E[C - 1]);
        eoR = pick<T, C>(ck.E, role.iright < 0 ? 0 : role.iright);
        eoR1 = choose<T>(role.iright >= 1, pick<T, C>(ck.E, role.iright - 1), prevLast);
    }
    chunk_h<T, C, PLASMA, CPML>(ck, get_er(ck.E[0]), ch);
    chunk_e<T, C, PLASMA, CPML>(ck, get_hl(ck.H[C - 1]), ce);
    if (role.src_any) {
        const double sv = source_value((double)m * g.dt, g.src_tau, g.src_t0, g.src_amp);
        if (role.isrc >= 0) put<T, C>(ck.E, role.isrc, add_source<T>(pick<T, C>(ck.E, role.isrc), sv));
    }
    chunk_j<T, C, PLASMA, CPML>(ck);
    if (role.left_any && role.ileft >= 0) {
        const T en1 = choose<T>(il, ck.E[2], ck.E[1]);
        const T v = (g.bc == 0) ? (T)(eo1 + (T)g.cm * (en1 - eo0)) : (T)0;
        if (il) ck.E[1] = v; else ck.E[0] = v;
    }
    if (role.right_any) {
        const T prevLast = shfl_up1(ck.E[C - 1]);
        const T enR1 = choose<T>(role.iright >= 1, pick<T, C>(ck.E, role.iright - 1), prevLast);
        if (role.iright >= 0)
            put<T, C>(ck.E, role.iright, (g.bc == 0) ? (T)(eoR1 + (T)g.cm * (enR1 - eoR)) : (T)0);
    }
}

}  // namespace fdtdp

namespace fdtdp {

// Role of this lane's chunk [k0, k0 + C) within grid b of n nodes.
__device__ __forceinline__ ChunkRole chunk_role(const Grids &g, int b, int64_t n, int64_t k0,
                                                int64_t wave_lo, int64_t wave_hi, int C)
{
    ChunkRole r;
    const int64_t s = g.src[b];
    r.src_any = s >= wave_lo && s < wave_hi;
    r.isrc = (s >= k0 && s < k0 + C) ? (int)(s - k0) : -1;
    r.left_any = wave_lo <= 0;
    r.ileft = (k0 <= 0 && k0 + C > 0) ? (int)(-k0) : -1;
    r.right_any = n - 1 >= wave_lo && n - 1 < wave_hi;
    r.iright = (n - 1 >= k0 && n - 1 < k0 + C) ? (int)(n - 1 - k0) : -1;
    return r;
}

// Probe samples of the lane's chunk for one step.
template <typename T, int C>
__device__ __forceinline__ void chunk_probes(const Grids &g, int b, int64_t k0, int64_t out_lo,
                                             int64_t out_hi, const T (&E)[C], int slot)
{
    for (int p = 0; p < g.P; ++p) {
        const int64_t q = g.probe[(int64_t)b * g.P + p];
        if (q >= out_lo && q < out_hi && q >= k0 && q < k0 + C)
            g.samp[((int64_t)b * g.P + p) * g.SB + slot] = (double)pick<T, C>(E, (int)(q - k0));
    }
}

// Block index remapped so that each XCD (workgroups are dealt round-robin to
// the 8 XCDs) receives a contiguous range of tiles and neighbouring tiles
// share an L2.
__device__ __forceinline__ int64_t xcd_block(int64_t bid, int64_t nblk)
{
    const int64_t q = nblk / 8, r = nblk % 8;
    const int64_t x = bid % 8, j = bid / 8;
    return x * q + (x < r ? x : r) + j;
}

template <typename T, int C, int KLASS>
__global__ __launch_bounds__(256) void k_tiled(Grids g, State<T> s, int cur, const Tile *tiles,
                                               int64_t ntiles, int nsteps, int64_t m0, int slot0)
{
    // class 0: vacuum tiles; 1: tiles with plasma; 2: tiles touching a CPML
    // layer (which may also hold plasma further in)
    constexpr bool PLASMA = KLASS >= 1;
    constexpr bool CPML = KLASS == 2;
    const int lane = threadIdx.x & 63;
    const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
    const int64_t t = blk * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (t >= ntiles) return;
    const Tile tl = tiles[t];
    const int b = tl.grid;
    const int64_t off = g.off[b], n = g.n[b];
    const int64_t k0 = (int64_t)tl.lo + (int64_t)lane * C;
    const int64_t wave_hi = (int64_t)tl.lo + 64LL * C;
    Chunk<T, C, PLASMA, CPML> ck;
    chunk_load<T, C, PLASMA, CPML>(ck, g, s, cur, b, off, n, k0, tl.hi);
    ChunkRole role = chunk_role(g, b, n, k0, tl.lo, tl.hi, C);
    const bool probes = (tl.flags & TILE_PROBE) != 0;
    auto er = [](T e0) { return shfl_down1(e0); };
    auto hl = [](T h) { return shfl_up1(h); };
    if (!(role.left_any || role.right_any || role.src_any || probes)) {
        // two steps per trip: the loop-carried E copies then alternate
        // registers instead of being moved back every step
        int st = 0;
        for (; st + 2 <= nsteps; st += 2) {
            chunk_step_plain<T, C, PLASMA, CPML>(ck, g, er, hl);
            chunk_step_plain<T, C, PLASMA, CPML>(ck, g, er, hl);
        }
        if (st < nsteps) chunk_step_plain<T, C, PLASMA, CPML>(ck, g, er, hl);
    } else {
        for (int st = 0; st < nsteps; ++st) {
            chunk_step<T, C, PLASMA, CPML>(ck, g, role, m0 + st + 1, er, hl);
            if (probes) chunk_probes<T, C>(g, b, k0, tl.out_lo, tl.out_hi, ck.E, slot0 + st);
        }
    }
    (void)wave_hi;
    chunk_store<T, C, PLASMA, CPML>(ck, g, s, cur ^ 1, b, off, n, k0, tl.out_lo, tl.out_hi);
}

// Workgroup tiles: one tile of WAVES * 64 * C nodes per workgroup, wave w
// holding the w-th run of 64*C nodes.  Edge values cross waves through LDS
// (two barriers per step, as in k_resident), so only the tile's two ends
// carry a halo.  Every wave takes both exchanges once per step on either
// path, so the barrier counts match.  The tile builder keeps node n-1 off
// the first node of a wave (the Mur end reads its left neighbour with an
// in-wave move).
template <typename T, int C, int KLASS, int WAVES>
__global__ __launch_bounds__(WAVES * 64) void k_tiledw(Grids g, State<T> s, int cur, const Tile *tiles,
                                                       int64_t ntiles, int nsteps, int64_t m0, int slot0)
{
    constexpr bool PLASMA = KLASS >= 1;
    constexpr bool CPML = KLASS == 2;
    __shared__ T ldsE[WAVES];
    __shared__ T ldsH[WAVES];
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int64_t t = xcd_block(blockIdx.x, gridDim.x);
    if (t >= ntiles) return;                  // whole workgroup: no barrier is left waiting
    const Tile tl = tiles[t];
    const int b = tl.grid;
    const int64_t off = g.off[b], n = g.n[b];
    const int64_t wave_lo = (int64_t)tl.lo + (int64_t)w * 64 * C;
    const int64_t wave_hi = wave_lo + 64LL * C < tl.hi ? wave_lo + 64LL * C : tl.hi;
    const int64_t k0 = wave_lo + (int64_t)lane * C;
    Chunk<T, C, PLASMA, CPML> ck;
    chunk_load<T, C, PLASMA, CPML>(ck, g, s, cur, b, off, n, k0, tl.hi);
    ChunkRole role = chunk_role(g, b, n, k0, wave_lo, wave_hi > wave_lo ? wave_hi : wave_lo, C);
    const bool probes = (tl.flags & TILE_PROBE) != 0;
    auto er = [&](T e0) {
        if (lane == 0) ldsE[w] = e0;
        __syncthreads();
        T v = shfl_down1(e0);
        if (lane == 63) v = (w + 1 < WAVES) ? ldsE[w + 1] : (T)0;
        return v;
    };
    auto hl = [&](T h) {
        if (lane == 63) ldsH[w] = h;
        __syncthreads();
        T v = shfl_up1(h);
        if (lane == 0) v = (w > 0) ? ldsH[w - 1] : (T)0;
        return v;
    };
    if (!(role.left_any || role.right_any || role.src_any || probes)) {
        for (int st = 0; st < nsteps; ++st) chunk_step_plain<T, C, PLASMA, CPML>(ck, g, er, hl);
    } else {
        for (int st = 0; st < nsteps; ++st) {
            chunk_step<T, C, PLASMA, CPML>(ck, g, role, m0 + st + 1, er, hl);
            if (probes) chunk_probes<T, C>(g, b, k0, tl.out_lo, tl.out_hi, ck.E, slot0 + st);
        }
    }
    chunk_store<T, C, PLASMA, CPML>(ck, g, s, cur ^ 1, b, off, n, k0, tl.out_lo, tl.out_hi);
}

template <typename T, int C, int WAVES>
void launch_tiledw_c(const Grids &g, State<T> &s, int cur, const Tile *tiles, int64_t ntiles, int klass,
                     int nsteps, int64_t m0, int slot0, hipStream_t st)
{
    const dim3 grid((unsigned)ntiles), blk(WAVES * 64);
    if (klass == 0)
        hipLaunchKernelGGL((k_tiledw<T, C, 0, WAVES>), grid, blk, 0, st, g, s, cur, tiles, ntiles, nsteps, m0,
                           slot0);
    else if (klass == 1)
        hipLaunchKernelGGL((k_tiledw<T, C, 1, WAVES>), grid, blk, 0, st, g, s, cur, tiles, ntiles, nsteps, m0,
                           slot0);
    else
        hipLaunchKernelGGL((k_tiledw<T, C, 2, WAVES>), grid, blk, 0, st, g, s, cur, tiles, ntiles, nsteps, m0,
                           slot0);
}

template <typename T, int WAVES>
void launch_tiledw_w(const Grids &g, State<T> &s, int cur, const Tile *tiles, int64_t ntiles, int klass,
                     int C, int nsteps, int64_t m0, int slot0, hipStream_t st)
{
    switch (C) {
    case 4: launch_tiledw_c<T, 4, WAVES>(g, s, cur, tiles, ntiles, klass, nsteps, m0, slot0, st); break;
    default: launch_tiledw_c<T, 8, WAVES>(g, s, cur, tiles, ntiles, klass, nsteps, m0, slot0, st); break;
    }
}

template <typename T, int C>
void launch_tiled_c(const Grids &g, State<T> &s, int cur, const Tile *tiles, int64_t ntiles,
                    int klass, int nsteps, int64_t m0, int slot0, hipStream_t st)
{
    const unsigned nb = (unsigned)((ntiles + 3) / 4);
    if (klass == 0)
        hipLaunchKernelGGL((k_tiled<T, C, 0>), dim3(nb), dim3(256), 0, st, g, s, cur, tiles, ntiles,
                           nsteps, m0, slot0);
    else if (klass == 1)
        hipLaunchKernelGGL((k_tiled<T, C, 1>), dim3(nb), dim3(256), 0, st, g, s, cur, tiles, ntiles,
                           nsteps, m0, slot0);
    else
        hipLaunchKernelGGL((k_tiled<T, C, 2>), dim3(nb), dim3(256), 0, st, g, s, cur, tiles, ntiles,
                           nsteps, m0, slot0);
}

template <typename T>
void launch_tiled(const Grids &g, State<T> &s, int cur, const Tile *tiles, int64_t ntiles, int klass,
                  int C, int nsteps, int64_t m0, int slot0, hipStream_t st, int waves)
{
    if (waves == 2) return launch_tiledw_w<T, 2>(g, s, cur, tiles, ntiles, klass, C, nsteps, m0, slot0, st);
    if (waves == 4) return launch_tiledw_w<T, 4>(g, s, cur, tiles, ntiles, klass, C, nsteps, m0, slot0, st);
    if (waves == 8) return launch_tiledw_w<T, 8>(g, s, cur, tiles, ntiles, klass, C, nsteps, m0, slot0, st);
    switch (C) {
    case 4: launch_tiled_c<T, 4>(g, s, cur, tiles, ntiles, klass, nsteps, m0, slot0, st); break;
    case 8: launch_tiled_c<T, 8>(g, s, cur, tiles, ntiles, klass, nsteps, m0, slot0, st); break;
    case 12: launch_tiled_c<T, 12>(g, s, cur, tiles, ntiles, klass, nsteps, m0, slot0, st); break;
    default: launch_tiled_c<T, 16>(g, s, cur, tiles, ntiles, klass, nsteps, m0, slot0, st); break;
    }
}

template void launch_tiled<float>(const Grids &, State<float> &, int, const Tile *, int64_t, int, int,
                                  int, int64_t, int, hipStream_t, int);
template void launch_tiled<double>(const Grids &, State<double> &, int, const Tile *, int64_t, int,
                                   int, int, int64_t, int, hipStream_t, int);

// ------------------------------------------------------------- resident

// One workgroup per bin of grids; slots[bin*WAVES + w] says which grid wave w
// holds.  Edge values cross waves through LDS: two barriers per step, taken by
// every wave of the workgroup (idle waves included) so the count matches.
template <typename T, int C, int WAVES>
__global__ __launch_bounds__(WAVES * 64) void k_resident(Grids g, State<T> s, int cur, int out,
                                                         const ResidentSlot *slots, int nsteps,
                                                         int64_t m0, int slot0)
{
    __shared__ T ldsE[WAVES];
    __shared__ T ldsH[WAVES];
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const ResidentSlot sl = slots[(int64_t)blockIdx.x * WAVES + w];
    const bool active = sl.grid >= 0;
    const int b = active ? sl.grid : 0;
    const int64_t off = g.off[b], n = active ? g.n[b] : 0;
    const int wi = w - sl.first_wave;                       // wave index within the grid
    // a grid whose node n-1 would open a wave is held one position to the
    // right (sl.shift = 1) so that nodes n-2 and n-1 share a lane
    const int64_t wave_lo = (int64_t)wi * 64 * C - sl.shift;
    const int64_t wave_hi = active ? (wave_lo + 64LL * C < n ? wave_lo + 64LL * C : n) : 0;
    const int64_t k0 = wave_lo + (int64_t)lane * C;
    const bool has_next = active && wi + 1 < sl.nwaves;
    const bool has_prev = active && wi > 0;
    Chunk<T, C, true, false> ck;
    if (active) chunk_load<T, C, true, false>(ck, g, s, cur, b, off, n, k0, n);
    else {
#pragma unroll
        for (int i = 0; i < C; ++i) {
            ck.E[i] = ck.H[i] = (T)0;
            ck.J[i] = ck.Ed[i] = 0.0;
        }
        ck.pmask = 0;
    }
    ChunkRole role = active ? chunk_role(g, b, n, k0, wave_lo < 0 ? 0 : wave_lo, wave_hi, C)
                            : ChunkRole{-1, -1, -1, false, false, false};
    for (int st = 0; st < nsteps; ++st) {
        auto get_er = [&](T e0) {
            if (lane == 0) ldsE[w] = e0;
            __syncthreads();
            T v = shfl_down1(e0);
            if (lane == 63) v = has_next ? ldsE[w + 1] : (T)0;
            return v;
        };
        auto get_hl = [&](T hl) {
            if (lane == 63) ldsH[w] = hl;
            __syncthreads();
            T v = shfl_up1(hl);
            if (lane == 0) v = has_prev ? ldsH[w - 1] : (T)0;
            return v;
        };
        chunk_step<T, C, true, false>(ck, g, role, m0 + st + 1, get_er, get_hl);
        if (active) chunk_probes<T, C>(g, b, k0, wave_lo < 0 ? 0 : wave_lo, wave_hi, ck.E, slot0 + st);
    }
    if (active) chunk_store<T, C, true, false>(ck, g, s, out, b, off, n, k0, 0, n);
}

template <typename T>
void launch_resident(const Grids &g, State<T> &s, int cur, int out, const ResidentSlot *slots, int64_t nbins,
                     int waves_per_wg, int C, int nsteps, int64_t m0, int slot0, hipStream_t st)
{
    (void)C;
    (void)waves_per_wg;   // 8 waves: 512 threads keep the per-node coefficients in VGPRs
    hipLaunchKernelGGL((k_resident<T, 8, 8>), dim3((unsigned)nbins), dim3(8 * 64), 0, st, g, s,
                       cur, out, slots, nsteps, m0, slot0);
}

template void launch_resident<float>(const Grids &, State<float> &, int, int, const ResidentSlot *, int64_t,
                                     int, int, int, int64_t, int, hipStream_t);
template void launch_resident<double>(const Grids &, State<double> &, int, int, const ResidentSlot *,
                                      int64_t, int, int, int, int64_t, int, hipStream_t);

int resident_max_nodes(int C, int waves) { return 64 * C * waves; }

}  // namespace fdtdp
