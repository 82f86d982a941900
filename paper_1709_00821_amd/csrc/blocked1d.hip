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

// Where a grid's special nodes sit in one wave's span of 64*C nodes: a
// node at position pos from the wave's first node is register pos % C of
// lane pos / C.  The values are the same in every lane (read through
// readfirstlane), so the register selects below run on scalar conditions.
// A lane of -1 means the wave does not hold the node.
struct WaveRole {
    int src_lane, src_reg;       // the source node
    int left_lane, left_reg;     // node 0: lane 0, register 0 or 1 (a wave never starts left of node -1)
    int right_lane, right_reg;   // node n-1: never register 0 of lane 0 (see the tile builder)
};

__device__ __forceinline__ int uniform(int64_t v) { return __builtin_amdgcn_readfirstlane((int)v); }

template <int C>
__device__ __forceinline__ WaveRole wave_role(const Grids &g, int b, int64_t n, int64_t wave_lo, int64_t wave_hi)
{
    const int64_t s = g.src[b];
    const int64_t ps = (s >= 0 && s >= wave_lo && s < wave_hi) ? s - wave_lo : -1;
    const int64_t pl = (wave_lo <= 0 && 0 < wave_hi) ? -wave_lo : -1;
    const int64_t pr = (n - 1 >= wave_lo && n - 1 < wave_hi) ? n - 1 - wave_lo : -1;
    WaveRole r;
    r.src_lane = uniform(ps >= 0 ? ps / C : -1);
    r.src_reg = uniform(ps >= 0 ? ps % C : 0);
    r.left_lane = uniform(pl >= 0 ? 0 : -1);
    r.left_reg = uniform(pl >= 0 ? pl : 0);
    r.right_lane = uniform(pr >= 0 ? pr / C : -1);
    r.right_reg = uniform(pr >= 0 ? pr % C : 1);
    return r;
}

__device__ __forceinline__ bool has_role(const WaveRole &r)
{
    return r.src_lane >= 0 || r.left_lane >= 0 || r.right_lane >= 0;
}

// v[i] for a wave-uniform i in [0, C).  The registers are gathered into one
// vector value and indexed there, which gfx950 code generation turns into
// C - 1 selects on scalar conditions.  (Selecting between the array elements
// directly would be folded into one load through a selected address and force
// the array into scratch memory.)
template <typename T, int C>
__device__ __forceinline__ T upick(const T (&v)[C], int i)
{
    typedef T vec __attribute__((ext_vector_type(C)));
    vec x;
#pragma unroll
    for (int j = 0; j < C; ++j) x[j] = v[j];
    return x[i];
}

// v[i] = x in the lanes where `here` holds (i wave-uniform).
template <typename T, int C>
__device__ __forceinline__ void uput(T (&v)[C], int i, bool here, T x)
{
#pragma unroll
    for (int j = 0; j < C; ++j) v[j] = (here && i == j) ? x : v[j];
}

__device__ __forceinline__ double readlane_d(double x, int l)
{
    const int2 v = __builtin_bit_cast(int2, x);
    return __builtin_bit_cast(double, make_int2(__builtin_amdgcn_readlane(v.x, l),
                                                __builtin_amdgcn_readlane(v.y, l)));
}

// The end values the Mur updates read, E^n at nodes 0, 1 and n-1, n-2, held
// from one step to the next: each equals what the previous step wrote (the
// end node) or read (its neighbour, which later sub-steps of that step leave
// alone).  Meaningful only in the lane holding the end.
template <typename T>
struct EndCarry {
    T e0, e1, eR, eR1;
};

template <typename T, int C>
__device__ __forceinline__ void ends_init(const T (&E)[C], const WaveRole &r, EndCarry<T> &c)
{
    c.e0 = r.left_reg ? E[1] : E[0];
    c.e1 = r.left_reg ? E[2] : E[1];
    const int ir = r.right_reg;
    c.eR = upick<T, C>(E, ir);
    c.eR1 = ir ? upick<T, C>(E, ir - 1) : shfl_up1(E[C - 1]);
}

// One full time step of a wave holding a grid end, the source or a probe: H,
// E, the source (added to E^{n+1}, eq.(15), before the J update), J, then the
// ends (first-order Mur, or PEC E = 0).  sv: the source value of this step.
// Every part runs in every such wave, as selects whose lane condition is
// false where the wave does not hold the node: no branch, so the registers
// need no merging copies.
template <typename T, int C, bool PLASMA, bool CPML, typename GetEr, typename GetHl>
__device__ __forceinline__ void chunk_step(Chunk<T, C, PLASMA, CPML> &ck, const Grids &g,
                                           const WaveRole &r, int lane, EndCarry<T> &c, double sv,
                                           GetEr get_er, GetHl get_hl)
{
    chunk_h<T, C, PLASMA, CPML>(ck, get_er(ck.E[0]), (T)g.ch);
    chunk_e<T, C, PLASMA, CPML>(ck, get_hl(ck.H[C - 1]), (T)g.ce);
    uput<T, C>(ck.E, r.src_reg, lane == r.src_lane, add_source<T>(upick<T, C>(ck.E, r.src_reg), sv));
    chunk_j<T, C, PLASMA, CPML>(ck);
    const bool mur = g.bc == 0;
    {
        const T en1 = r.left_reg ? ck.E[2] : ck.E[1];
        const T v = mur ? (T)(c.e1 + (T)g.cm * (en1 - c.e0)) : (T)0;
        const bool here = lane == r.left_lane;
        ck.E[0] = (here && !r.left_reg) ? v : ck.E[0];
        ck.E[1] = (here && r.left_reg) ? v : ck.E[1];
        c.e0 = v;
        c.e1 = en1;
    }
    {
        const int ir = r.right_reg;
        const T prev = shfl_up1(ck.E[C - 1]);
        const T left1 = upick<T, C>(ck.E, ir > 0 ? ir - 1 : 0);
        const T en1 = ir > 0 ? left1 : prev;
        const T v = mur ? (T)(c.eR1 + (T)g.cm * (en1 - c.eR)) : (T)0;
        uput<T, C>(ck.E, ir, lane == r.right_lane, v);
        c.eR = v;
        c.eR1 = en1;
    }
}

}  // namespace fdtdp

namespace fdtdp {

// The probes a wave samples: those of grid b at nodes in [lo, hi) (inside
// the wave's span).  The first two are kept as wave-uniform lane, register
// and sample-row offset; a wave with more walks the probe list every step.
struct WaveProbes {
    int n;                 // probes in range
    int lane[2], reg[2];   // where the probe node sits in the wave
    int64_t row[2];        // (b * P + p) * SB: the probe's row of the sample buffer
};

template <int C>
__device__ __forceinline__ WaveProbes wave_probes_find(const Grids &g, int b, int64_t wave_lo, int64_t lo,
                                                      int64_t hi)
{
    int n = 0;
    int64_t q0 = 0, q1 = 0, r0 = 0, r1 = 0;
    for (int p = 0; p < g.P; ++p) {
        const int64_t q = g.probe[(int64_t)b * g.P + p];
        if (q >= lo && q < hi) {
            const int64_t row = ((int64_t)b * g.P + p) * g.SB;
            if (n == 0) { q0 = q - wave_lo; r0 = row; }
            if (n == 1) { q1 = q - wave_lo; r1 = row; }
            ++n;
        }
    }
    WaveProbes w;
    w.n = uniform(n);
    w.lane[0] = uniform(q0 / C);
    w.reg[0] = uniform(q0 % C);
    w.lane[1] = uniform(q1 / C);
    w.reg[1] = uniform(q1 % C);
    w.row[0] = (int64_t)__builtin_amdgcn_readfirstlane((int)r0) |
               ((int64_t)__builtin_amdgcn_readfirstlane((int)(r0 >> 32)) << 32);
    w.row[1] = (int64_t)__builtin_amdgcn_readfirstlane((int)r1) |
               ((int64_t)__builtin_amdgcn_readfirstlane((int)(r1 >> 32)) << 32);
    return w;
}

template <typename T, int C>
__device__ __forceinline__ void wave_probe_store(const Grids &g, int lane_p, int reg, int64_t row, int lane,
                                                 const T (&E)[C], int slot)
{
    const T v = upick<T, C>(E, reg);
    if (lane == lane_p) g.samp[row + slot] = (double)v;
}

// Samples of one step (after the step's ends), one store per probe: the
// path for a wave that holds more than two probes.
template <typename T, int C>
__device__ __forceinline__ void wave_probes(const Grids &g, int b, int64_t wave_lo, int64_t lo, int64_t hi,
                                            int lane, const T (&E)[C], int slot)
{
    for (int p = 0; p < g.P; ++p) {
        const int64_t q = g.probe[(int64_t)b * g.P + p];
        if (q >= lo && q < hi) {
            const int pos = uniform(q - wave_lo);
            wave_probe_store<T, C>(g, pos / C, pos % C, ((int64_t)b * g.P + p) * g.SB, lane, E, slot);
        }
    }
}

// nsteps full steps of a wave that holds a grid end, the source or a probe
// (sample slots slot0 .. slot0 + nsteps - 1 of the window), in runs of up to
// 64 steps.  The only load is at the start of a run: the source values of its
// steps, one per lane of the window's table, broadcast from lane st.  Inside a
// run the wave issues nothing but the probe stores, which it never waits on.
// (Every cross-lane read here takes a value all lanes computed: a value
// computed only in some lanes would be stale in the lane that is read.)
template <typename T, int C, bool PLASMA, bool CPML, typename GetEr, typename GetHl, typename Post>
__device__ __forceinline__ void run_role(Chunk<T, C, PLASMA, CPML> &ck, const Grids &g, const WaveRole &r,
                                         const WaveProbes &wp, int lane, int b, int64_t wave_lo, int64_t plo,
                                         int64_t phi, int nsteps, int slot0, GetEr er, GetHl hl, Post post)
{
    EndCarry<T> c;
    ends_init<T, C>(ck.E, r, c);
    for (int base = 0; base < nsteps; base += 64) {
        const int cnt = nsteps - base < 64 ? nsteps - base : 64;
        const int slot = slot0 + base;
        double svl = 0.0;
        if (r.src_lane >= 0) {
            const int i = slot + lane;
            svl = g.srcv[i < g.SB ? i : g.SB - 1];
        }
        auto one = [&](int st) {
            const double sv = (r.src_lane >= 0) ? readlane_d(svl, st) : 0.0;
            chunk_step<T, C, PLASMA, CPML>(ck, g, r, lane, c, sv, er, hl);
            post(base + st);
            if (wp.n > 2) {
                wave_probes<T, C>(g, b, wave_lo, plo, phi, lane, ck.E, slot + st);
            } else {
                if (wp.n > 0) wave_probe_store<T, C>(g, wp.lane[0], wp.reg[0], wp.row[0], lane, ck.E, slot + st);
                if (wp.n > 1) wave_probe_store<T, C>(g, wp.lane[1], wp.reg[1], wp.row[1], lane, ck.E, slot + st);
            }
        };
        int st = 0;
        for (; st + 2 <= cnt; st += 2) {
            one(st);
            one(st + 1);
        }
        if (st < cnt) one(st);
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

template <typename T, int C, int KLASS, bool ROLES>
__global__ __launch_bounds__(256) void k_tiled(Grids g, State<T> s, int cur, const Tile *tiles,
                                               int64_t ntiles, int nsteps, int slot0)
{
    // class 0: vacuum tiles; 1: tiles with plasma; 2: tiles touching a CPML
    // layer (which may also hold plasma further in).  ROLES: the tiles hold a
    // grid end, the source or a probe (a separate instantiation, so that the
    // bulk tiles' register budget is that of the plain step alone)
    constexpr bool PLASMA = KLASS >= 1;
    constexpr bool CPML = KLASS == 2;
    const int lane = threadIdx.x & 63;
    const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
    const int64_t t = blk * (blockDim.x >> 6) + uniform(threadIdx.x >> 6);
    if (t >= ntiles) return;
    const Tile tl = tiles[t];
    const int b = tl.grid;
    const int64_t off = g.off[b], n = g.n[b];
    const int64_t k0 = (int64_t)tl.lo + (int64_t)lane * C;
    Chunk<T, C, PLASMA, CPML> ck;
    chunk_load<T, C, PLASMA, CPML>(ck, g, s, cur, b, off, n, k0, tl.hi);
    auto er = [](T e0) { return shfl_down1(e0); };
    auto hl = [](T h) { return shfl_up1(h); };
    if constexpr (!ROLES) {
        // two steps per trip: the loop-carried E copies then alternate
        // registers instead of being moved back every step
        int st = 0;
        for (; st + 2 <= nsteps; st += 2) {
            chunk_step_plain<T, C, PLASMA, CPML>(ck, g, er, hl);
            chunk_step_plain<T, C, PLASMA, CPML>(ck, g, er, hl);
        }
        if (st < nsteps) chunk_step_plain<T, C, PLASMA, CPML>(ck, g, er, hl);
    } else {
        const WaveRole role = wave_role<C>(g, b, n, tl.lo, tl.hi);
        WaveProbes wp;
        wp.n = 0;
        if (tl.flags & TILE_PROBE) wp = wave_probes_find<C>(g, b, tl.lo, tl.out_lo, tl.out_hi);
        run_role<T, C, PLASMA, CPML>(ck, g, role, wp, lane, b, tl.lo, tl.out_lo, tl.out_hi, nsteps, slot0, er,
                                     hl, [](int) {});
    }
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
                                                       int64_t ntiles, int nsteps, int slot0)
{
    constexpr bool PLASMA = KLASS >= 1;
    constexpr bool CPML = KLASS == 2;
    __shared__ T ldsE[WAVES];
    __shared__ T ldsH[WAVES];
    const int lane = threadIdx.x & 63;
    const int w = uniform(threadIdx.x >> 6);
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
    const WaveRole role = wave_role<C>(g, b, n, wave_lo, wave_hi > wave_lo ? wave_hi : wave_lo);
    const bool probes = (tl.flags & TILE_PROBE) != 0;
    // probes this wave samples: tile outputs inside the wave's span
    const int64_t plo = tl.out_lo > wave_lo ? tl.out_lo : wave_lo;
    const int64_t phi = tl.out_hi < wave_hi ? tl.out_hi : wave_hi;
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
    WaveProbes wp;
    wp.n = 0;
    if (probes && plo < phi) wp = wave_probes_find<C>(g, b, wave_lo, plo, phi);
    if (!has_role(role) && wp.n == 0) {
        for (int st = 0; st < nsteps; ++st) chunk_step_plain<T, C, PLASMA, CPML>(ck, g, er, hl);
    } else {
        run_role<T, C, PLASMA, CPML>(ck, g, role, wp, lane, b, wave_lo, plo, phi, nsteps, slot0, er, hl,
                                     [](int) {});
    }
    chunk_store<T, C, PLASMA, CPML>(ck, g, s, cur ^ 1, b, off, n, k0, tl.out_lo, tl.out_hi);
}

template <typename T, int C, int WAVES>
void launch_tiledw_c(const Grids &g, State<T> &s, int cur, const Tile *tiles, int64_t ntiles, int klass,
                     int nsteps, int slot0, hipStream_t st)
{
    const dim3 grid((unsigned)ntiles), blk(WAVES * 64);
    // class 3 (role tiles) takes the plasma kernel, which holds both paths
    if (klass == 0)
        hipLaunchKernelGGL((k_tiledw<T, C, 0, WAVES>), grid, blk, 0, st, g, s, cur, tiles, ntiles, nsteps,
                           slot0);
    else if (klass == 2)
        hipLaunchKernelGGL((k_tiledw<T, C, 2, WAVES>), grid, blk, 0, st, g, s, cur, tiles, ntiles, nsteps,
                           slot0);
    else
        hipLaunchKernelGGL((k_tiledw<T, C, 1, WAVES>), grid, blk, 0, st, g, s, cur, tiles, ntiles, nsteps,
                           slot0);
}

template <typename T, int WAVES>
void launch_tiledw_w(const Grids &g, State<T> &s, int cur, const Tile *tiles, int64_t ntiles, int klass,
                     int C, int nsteps, int slot0, hipStream_t st)
{
    switch (C) {
    case 4: launch_tiledw_c<T, 4, WAVES>(g, s, cur, tiles, ntiles, klass, nsteps, slot0, st); break;
    default: launch_tiledw_c<T, 8, WAVES>(g, s, cur, tiles, ntiles, klass, nsteps, slot0, st); break;
    }
}

template <typename T, int C>
void launch_tiled_c(const Grids &g, State<T> &s, int cur, const Tile *tiles, int64_t ntiles,
                    int klass, int nsteps, int slot0, hipStream_t st)
{
    const unsigned nb = (unsigned)((ntiles + 3) / 4);
    if (klass == 0)
        hipLaunchKernelGGL((k_tiled<T, C, 0, false>), dim3(nb), dim3(256), 0, st, g, s, cur, tiles, ntiles,
                           nsteps, slot0);
    else if (klass == 1)
        hipLaunchKernelGGL((k_tiled<T, C, 1, false>), dim3(nb), dim3(256), 0, st, g, s, cur, tiles, ntiles,
                           nsteps, slot0);
    else if (klass == 2)
        hipLaunchKernelGGL((k_tiled<T, C, 2, true>), dim3(nb), dim3(256), 0, st, g, s, cur, tiles, ntiles,
                           nsteps, slot0);
    else   // role tiles, vacuum or plasma: the plasma step reproduces the vacuum one
        hipLaunchKernelGGL((k_tiled<T, C, 1, true>), dim3(nb), dim3(256), 0, st, g, s, cur, tiles, ntiles,
                           nsteps, slot0);
}

template <typename T>
void launch_tiled(const Grids &g, State<T> &s, int cur, const Tile *tiles, int64_t ntiles, int klass,
                  int C, int nsteps, int slot0, hipStream_t st, int waves)
{
    if (waves == 2) return launch_tiledw_w<T, 2>(g, s, cur, tiles, ntiles, klass, C, nsteps, slot0, st);
    if (waves == 4) return launch_tiledw_w<T, 4>(g, s, cur, tiles, ntiles, klass, C, nsteps, slot0, st);
    if (waves == 8) return launch_tiledw_w<T, 8>(g, s, cur, tiles, ntiles, klass, C, nsteps, slot0, st);
    switch (C) {
    case 4: launch_tiled_c<T, 4>(g, s, cur, tiles, ntiles, klass, nsteps, slot0, st); break;
    case 8: launch_tiled_c<T, 8>(g, s, cur, tiles, ntiles, klass, nsteps, slot0, st); break;
    case 12: launch_tiled_c<T, 12>(g, s, cur, tiles, ntiles, klass, nsteps, slot0, st); break;
    default: launch_tiled_c<T, 16>(g, s, cur, tiles, ntiles, klass, nsteps, slot0, st); break;
    }
}

template void launch_tiled<float>(const Grids &, State<float> &, int, const Tile *, int64_t, int, int,
                                  int, int, hipStream_t, int);
template void launch_tiled<double>(const Grids &, State<double> &, int, const Tile *, int64_t, int,
                                   int, int, int, hipStream_t, int);

// ------------------------------------------------------------ trace

// Forward recompute for the adjoint: the tiles of every grid advance nsteps
// steps from segment slot slot0 and store the state of their output nodes
// after every step into slots slot0 + 1 .. slot0 + nsteps (slot i at
// seg + i * slot_bytes: E [nodes], H at + arr_bytes, J (FP64) at + 2 arr_bytes).
// Same per-node functions as k_tiled, hence the forward run's bits.  Tiles
// read only slot slot0, which no tile of the launch writes.  Mur or PEC ends;
// no probes (g.P = 0); the source values come from g.srcv indexed by slot.
template <typename T, int C>
__global__ __launch_bounds__(256) void k_trace(Grids g, char *seg, int64_t slot_bytes, int64_t arr_bytes,
                                               const Tile *tiles, int64_t ntiles, int nsteps, int slot0)
{
    const int lane = threadIdx.x & 63;
    const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
    const int64_t t = blk * (blockDim.x >> 6) + uniform(threadIdx.x >> 6);
    if (t >= ntiles) return;
    const Tile tl = tiles[t];
    const int b = tl.grid;
    const int64_t off = g.off[b], n = g.n[b];
    const int64_t k0 = (int64_t)tl.lo + (int64_t)lane * C;
    auto slotE = [&](int i) { return (T *)(seg + (int64_t)i * slot_bytes); };
    auto slotH = [&](int i) { return (T *)(seg + (int64_t)i * slot_bytes + arr_bytes); };
    auto slotJ = [&](int i) { return (double *)(seg + (int64_t)i * slot_bytes + 2 * arr_bytes); };
    State<T> s0;
    s0.E[0] = slotE(slot0);
    s0.H[0] = slotH(slot0);
    s0.J[0] = slotJ(slot0);
    Chunk<T, C, true, false> ck;
    chunk_load<T, C, true, false>(ck, g, s0, 0, b, off, n, k0, tl.hi);
    auto er = [](T e0) { return shfl_down1(e0); };
    auto hl = [](T h) { return shfl_up1(h); };
    auto post = [&](int st) {
        const int i = slot0 + st + 1;
        store_chunk<T, C>(slotE(i) + off, k0, tl.out_lo, tl.out_hi, ck.E);
        store_chunk<T, C>(slotH(i) + off, k0, tl.out_lo, tl.out_hi < n ? tl.out_hi : n - 1, ck.H);
        store_chunk<double, C>(slotJ(i) + off, k0, tl.out_lo, tl.out_hi, ck.J);
    };
    const WaveRole role = wave_role<C>(g, b, n, tl.lo, tl.hi);
    if (!has_role(role)) {
        for (int st = 0; st < nsteps; ++st) {
            chunk_step_plain<T, C, true, false>(ck, g, er, hl);
            post(st);
        }
    } else {
        WaveProbes wp;
        wp.n = 0;
        run_role<T, C, true, false>(ck, g, role, wp, lane, b, tl.lo, tl.out_lo, tl.out_hi, nsteps, slot0, er, hl,
                                    post);
    }
}

template <typename T>
void launch_trace(const Grids &g, char *seg, int64_t slot_bytes, int64_t arr_bytes, const Tile *tiles,
                  int64_t ntiles, int nsteps, int slot0, hipStream_t st)
{
    hipLaunchKernelGGL((k_trace<T, kTraceCells / 64>), dim3((unsigned)((ntiles + 3) / 4)), dim3(256), 0, st, g, seg,
                       slot_bytes, arr_bytes, tiles, ntiles, nsteps, slot0);
}

template void launch_trace<float>(const Grids &, char *, int64_t, int64_t, const Tile *, int64_t, int, int,
                                  hipStream_t);
template void launch_trace<double>(const Grids &, char *, int64_t, int64_t, const Tile *, int64_t, int, int,
                                   hipStream_t);

// ------------------------------------------------------------ reverse

// Transposed steps of the adjoint on register tiles: lane holds C nodes of
// lambda_E, lambda_H, lambda_J (storage precision, as between the steps of
// the per-step kernel), the eleven coefficient and derivative values and the
// gradient of its nodes (FP64).  Reverse step m (lambda^{m+1} -> lambda^m),
// for interior nodes k, with es the adjoint of the E update's input, lHn the
// adjoint of H^{m+1/2}:
//   lEp = lambda_E (+ dL/dE^{m+1} at the probe node)
//   es  = lEp (+ cm lEp(0) at node 1, + cm lEp(n-1) at node n-2, Mur) + b2 lambda_J
//   lHn = lambda_H + CH(k+1) es(k+1) [k+1 <= n-2] - CH(k) es(k) [k >= 1]
//   lambda_J' = a lambda_J - CJ es
//   lambda_E' = CA es + b1 lambda_J + ch (lHn(k) - lHn(k-1)) (+ lEp(0) at 1, + lEp(n-1) at n-2)
//   grad += es (dCA E^m - dCJ J^m - dCH curl H^{m+1/2}) + lambda_J (db1 E^m + db2 E^{m+1})
// and at the end nodes lambda_E' = -cm lEp(k) +- ch lHn (Mur) or 0 (PEC).
// The expressions and their order are those of the per-step kernel, so the
// two give the same bits.  The stencil radius is one node per step, as in
// the forward step, so a tile with a kAdjHalo halo runs up to kAdjHalo steps.
// ROLE: the tile holds a grid end or the probe node (conditions evaluated per
// node); otherwise every held node is interior.
template <typename T, int C, bool ROLE>
__device__ __forceinline__ void adj_tile_steps(const Grids &g, const AdjTileArgs<T> &a, const Tile &tl, int b,
                                               int64_t off, int64_t n, int64_t k0, int lane, int64_t mtop,
                                               int nsteps, T (&lE)[C], T (&lH)[C], T (&lJ)[C],
                                               double (&gr)[C])
{
    const int64_t tot = a.total;
    double CA[C], CJ[C], CH[C], CHn[C], A[C], B1[C], B2[C], dCA[C], dCJ[C], dCH[C], dB1[C], dB2[C];
    load_chunk<double, C>(a.tab + 0 * tot + off, k0, tl.hi, CA);
    load_chunk<double, C>(a.tab + 1 * tot + off, k0, tl.hi, CJ);
    load_chunk<double, C>(a.tab + 2 * tot + off, k0, tl.hi, CH);
    load_chunk<double, C>(a.tab + 3 * tot + off, k0, tl.hi, A);
    load_chunk<double, C>(a.tab + 4 * tot + off, k0, tl.hi, B1);
    load_chunk<double, C>(a.tab + 5 * tot + off, k0, tl.hi, B2);
    load_chunk<double, C>(a.tab + 6 * tot + off, k0, tl.hi, dCA);
    load_chunk<double, C>(a.tab + 7 * tot + off, k0, tl.hi, dCJ);
    load_chunk<double, C>(a.tab + 8 * tot + off, k0, tl.hi, dCH);
    load_chunk<double, C>(a.tab + 9 * tot + off, k0, tl.hi, dB1);
    load_chunk<double, C>(a.tab + 10 * tot + off, k0, tl.hi, dB2);
    {
        const double nx = shfl_down1(CH[0]);
#pragma unroll
        for (int i = 0; i < C; ++i) CHn[i] = (i + 1 < C) ? CH[i + 1] : nx;
    }
    const bool mur = g.bc == 0;
    const double cm = g.cm, ch = g.ch;
    // the probe node, if this tile holds it (wave-uniform)
    const int64_t pc = g.probe[(int64_t)b * g.P + a.probe];
    const bool has_p = ROLE && pc >= tl.lo && pc < tl.hi;
    const int p_lane = uniform(has_p ? (pc - tl.lo) / C : -1), p_reg = uniform(has_p ? (pc - tl.lo) % C : 0);
    const int nn = (int)n;
    auto slotp = [&](int64_t m, int q) { return a.seg + (m - a.m0) * a.slot_bytes + q * a.arr_bytes; };
    // forward states E^m, J^m, H^{m+1/2}, E^{m+1} of the next step are loaded
    // one step ahead (E^{m+1} of step m-1 is this step's E^m)
    T ne0[C], nhh[C], ne1[C];
    double nj0[C];
    load_chunk<T, C>((const T *)slotp(mtop, 0) + off, k0, tl.hi, ne0);
    load_chunk<double, C>((const double *)slotp(mtop, 2) + off, k0, tl.hi, nj0);
    load_chunk<T, C>((const T *)slotp(mtop + 1, 1) + off, k0, tl.hi, nhh);
    load_chunk<T, C>((const T *)slotp(mtop + 1, 0) + off, k0, tl.hi, ne1);
    for (int st = 0; st < nsteps; ++st) {
        const int64_t m = mtop - st;
        T e0[C], hh[C], e1[C];
        double j0[C];
#pragma unroll
        for (int i = 0; i < C; ++i) {
            e0[i] = ne0[i];
            j0[i] = nj0[i];
            hh[i] = nhh[i];
            e1[i] = ne1[i];
        }
        if (st + 1 < nsteps) {
#pragma unroll
            for (int i = 0; i < C; ++i) ne1[i] = e0[i];
            load_chunk<T, C>((const T *)slotp(m - 1, 0) + off, k0, tl.hi, ne0);
            load_chunk<double, C>((const double *)slotp(m - 1, 2) + off, k0, tl.hi, nj0);
            load_chunk<T, C>((const T *)slotp(m, 1) + off, k0, tl.hi, nhh);
        }
        const double src = has_p ? a.gsrc[(int64_t)b * a.T_ + m] : 0.0;
        double lEp[C], es[C], lHn[C];
#pragma unroll
        for (int i = 0; i < C; ++i) {
            const double l = (double)lE[i];
            lEp[i] = (ROLE && lane == p_lane && i == p_reg) ? l + src : l;
        }
        double lEp0 = 0.0, lEpN = 0.0;
        if constexpr (ROLE) {
            // lEp at node 0 for node 1 (same lane: node 0 sits in register 0
            // or 1 of lane 0), at node n-1 for node n-2 (same lane, or the
            // next lane's register 0)
            const int r0 = uniform(tl.lo <= 0 ? -tl.lo : 0);
            lEp0 = upick<double, C>(lEp, r0);
            const int64_t pr = n - 1 - tl.lo;
            const int rr = uniform(pr >= 0 && pr < 64LL * C ? pr % C : 1);
            const double nx = shfl_down1(lEp[0]);
            const double own = upick<double, C>(lEp, rr);
            lEpN = (rr > 0) ? own : nx;
        }
#pragma unroll
        for (int i = 0; i < C; ++i) {
            double s = lEp[i];
            if constexpr (ROLE) {
                const int k = (int)(k0 + i);
                s = (mur && k == 1) ? s + cm * lEp0 : s;
                s = (mur && k == nn - 2) ? s + cm * lEpN : s;
            }
            es[i] = s + B2[i] * (double)lJ[i];
        }
        const double esn = shfl_down1(es[0]);
#pragma unroll
        for (int i = 0; i < C; ++i) {
            const double en = (i + 1 < C) ? es[i + 1] : esn;
            double s = (double)lH[i];
            if constexpr (ROLE) {
                const int k = (int)(k0 + i);
                s = (k + 1 <= nn - 2) ? s + CHn[i] * en : s;
                s = (k >= 1) ? s - CH[i] * es[i] : s;
            } else {
                s += CHn[i] * en;
                s -= CH[i] * es[i];
            }
            lHn[i] = s;
        }
        const double lHp = shfl_up1(lHn[C - 1]);
        const T hhp = shfl_up1(hh[C - 1]);
#pragma unroll
        for (int i = 0; i < C; ++i) {
            const double lhm = (i > 0) ? lHn[i - 1] : lHp;
            const double lj = (double)lJ[i];
            double nJ = A[i] * lj - CJ[i] * es[i];
            double nE = CA[i] * es[i] + B1[i] * lj + ch * (lHn[i] - lhm);
            const double curl = (double)hh[i] - (double)((i > 0) ? hh[i - 1] : hhp);
            const double e0d = (double)e0[i], e1d = (double)e1[i];
            const double gnew =
                gr[i] + (es[i] * (dCA[i] * e0d - dCJ[i] * j0[i] - dCH[i] * curl) + lj * (dB1[i] * e0d + dB2[i] * e1d));
            if constexpr (ROLE) {
                const int k = (int)(k0 + i);
                nE = (mur && k == 1) ? nE + lEp0 : nE;
                nE = (mur && k == nn - 2) ? nE + lEpN : nE;
                const bool end = k == 0 || k == nn - 1;
                const double nEe = mur ? -cm * lEp[i] + (k == 0 ? ch * lHn[i] : -ch * lhm) : 0.0;
                nE = end ? nEe : nE;
                nJ = end ? 0.0 : nJ;
                gr[i] = (k >= 1 && k <= nn - 2) ? gnew : gr[i];
            } else {
                gr[i] = gnew;
            }
            lE[i] = (T)nE;
            lJ[i] = (T)nJ;
            lH[i] = (T)lHn[i];
        }
    }
}

template <typename T, int C>
__global__ __launch_bounds__(256) void k_adj_tiled(Grids g, AdjTileArgs<T> a, const Tile *tiles, int64_t ntiles,
                                                   int64_t mtop, int nsteps)
{
    const int lane = threadIdx.x & 63;
    const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
    const int64_t t = blk * (blockDim.x >> 6) + uniform(threadIdx.x >> 6);
    if (t >= ntiles) return;
    const Tile tl = tiles[t];
    const int b = tl.grid;
    const int64_t off = g.off[b], n = g.n[b];
    const int64_t k0 = (int64_t)tl.lo + (int64_t)lane * C;
    T lE[C], lH[C], lJ[C];
    double gr[C];
    load_chunk<T, C>(a.lE + off, k0, tl.hi, lE);
    load_chunk<T, C>(a.lH + off, k0, tl.hi, lH);
    load_chunk<T, C>(a.lJ + off, k0, tl.hi, lJ);
    load_chunk<double, C>(a.grad + off, k0, tl.hi, gr);
    const int64_t pc = g.probe[(int64_t)b * g.P + a.probe];
    const bool role = tl.lo <= 0 || tl.hi >= n || (pc >= tl.lo && pc < tl.hi);
    if (role)
        adj_tile_steps<T, C, true>(g, a, tl, b, off, n, k0, lane, mtop, nsteps, lE, lH, lJ, gr);
    else
        adj_tile_steps<T, C, false>(g, a, tl, b, off, n, k0, lane, mtop, nsteps, lE, lH, lJ, gr);
    store_chunk<T, C>(a.nE + off, k0, tl.out_lo, tl.out_hi, lE);
    store_chunk<T, C>(a.nH + off, k0, tl.out_lo, tl.out_hi < n ? tl.out_hi : n - 1, lH);
    store_chunk<T, C>(a.nJ + off, k0, tl.out_lo, tl.out_hi, lJ);
    store_chunk<double, C>(a.grad + off, k0, tl.out_lo, tl.out_hi, gr);
}

template <typename T>
void launch_adj_tiled(const Grids &g, const AdjTileArgs<T> &a, const Tile *tiles, int64_t ntiles, int64_t mtop,
                      int nsteps, hipStream_t st)
{
    hipLaunchKernelGGL((k_adj_tiled<T, kAdjCells / 64>), dim3((unsigned)((ntiles + 3) / 4)), dim3(256), 0, st, g,
                       a, tiles, ntiles, mtop, nsteps);
}

template void launch_adj_tiled<float>(const Grids &, const AdjTileArgs<float> &, const Tile *, int64_t, int64_t,
                                      int, hipStream_t);
template void launch_adj_tiled<double>(const Grids &, const AdjTileArgs<double> &, const Tile *, int64_t, int64_t,
                                       int, hipStream_t);

// ------------------------------------------------------------- resident

// One workgroup per bin of grids; slots[bin*WAVES + w] says which grid wave w
// holds.  Edge values cross waves through LDS: two barriers per step, taken by
// every wave of the workgroup (idle waves included) so the count matches.
template <typename T, int C, int WAVES>
__global__ __launch_bounds__(WAVES * 64) void k_resident(Grids g, State<T> s, int cur, int out,
                                                         const ResidentSlot *slots, int nsteps,
                                                         int slot0)
{
    __shared__ T ldsE[WAVES];
    __shared__ T ldsH[WAVES];
    const int lane = threadIdx.x & 63;
    const int w = uniform(threadIdx.x >> 6);
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
    const WaveRole role = active ? wave_role<C>(g, b, n, wave_lo, wave_hi) : WaveRole{-1, 0, -1, 0, -1, 1};
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
    const int64_t plo = wave_lo < 0 ? 0 : wave_lo;
    WaveProbes wp;
    wp.n = 0;
    if (active) wp = wave_probes_find<C>(g, b, wave_lo, plo, wave_hi);
    // waves holding no end, source or probe take the plain step; both paths
    // cross the two barriers of get_er / get_hl once per step
    if (!has_role(role) && wp.n == 0) {
        for (int st = 0; st < nsteps; ++st) chunk_step_plain<T, C, true, false>(ck, g, get_er, get_hl);
    } else {
        run_role<T, C, true, false>(ck, g, role, wp, lane, b, wave_lo, plo, wave_hi, nsteps, slot0, get_er,
                                    get_hl, [](int) {});
    }
    if (active) chunk_store<T, C, true, false>(ck, g, s, out, b, off, n, k0, 0, n);
}

template <typename T>
void launch_resident(const Grids &g, State<T> &s, int cur, int out, const ResidentSlot *slots, int64_t nbins,
                     int waves_per_wg, int C, int nsteps, int slot0, hipStream_t st)
{
    (void)C;
    (void)waves_per_wg;   // 8 waves: 512 threads keep the per-node coefficients in VGPRs
    hipLaunchKernelGGL((k_resident<T, 8, 8>), dim3((unsigned)nbins), dim3(8 * 64), 0, st, g, s,
                       cur, out, slots, nsteps, slot0);
}

template void launch_resident<float>(const Grids &, State<float> &, int, int, const ResidentSlot *, int64_t,
                                     int, int, int, int, hipStream_t);
template void launch_resident<double>(const Grids &, State<double> &, int, int, const ResidentSlot *,
                                      int64_t, int, int, int, int, hipStream_t);

int resident_max_nodes(int C, int waves) { return 64 * C * waves; }

}  // namespace fdtdp
