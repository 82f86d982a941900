// Register-tile building blocks of the 1D kernels (gfx950): each lane holds
// C consecutive nodes of E, H (and J, coefficients in plasma, psi in CPML
// layers) in VGPRs; a wave holds 64*C consecutive nodes.  One time step
// needs two neighbour values per lane, moved with cross-lane DPP.  Used by
// the forward tile and resident kernels (blocked1d.hip) and the adjoint
// recompute and reverse kernels (adjoint1d.hip).
#ifndef FDTDP_TILE1D_H
#define FDTDP_TILE1D_H

#include <hip/hip_runtime.h>

#include "internal.h"

namespace fdtdp {

// ------------------------------------------------------------ chunk state

template <bool JF>
struct JType {
    typedef double type;
};
template <>
struct JType<true> {
    typedef float type;
};

// Register type of the field arithmetic for storage type T: FP64, except in
// the FP32 ablation (JF), whose every update runs in FP32.  FP32 storage with
// FP64 registers rounds E and H (and psi) to FP32 only where a launch stores
// them, not after every step: rounding the fields to FP32 after every step
// lets the rounding errors collect in the modes an open 1D grid does not
// damp (with first-order Mur ends a uniform offset of E or of H is a steady
// state), which dominates the reflection and transmission error at the low
// end of the band.
template <typename T, bool JF>
struct RegOf {
    typedef double type;
};
template <>
struct RegOf<float, true> {
    typedef float type;
};

// JF: the FP32 delta-form ablation of eq.(11) (J and its update in FP32).
template <typename T, int C, bool PLASMA, bool CPML, bool JF = false>
struct Chunk {
    typedef typename JType<JF>::type JT;
    typedef typename RegOf<T, JF>::type R;
    R E[C], H[C];
    JT J[PLASMA ? C : 1];          // Q = CJ (J - b2 E) in FP64 (the ablation: J itself, in FP32)
    JT Ed[JF && PLASMA ? C : 1];   // the ablation: E^n, the J update's E_old, kept across steps
    NodeCoef<R> cf[PLASMA ? C : 1];   // eH (and in the ablation eJ) held negated (see chunk_load)
    float jc[JF && PLASMA ? 3 * C : 1];   // JF: a-1, b1, b2 of each node rounded to FP32
    R nch, nce;                    // -dt/(mu0 dz), -dt/(eps0 dz)
    R pE[CPML ? C : 1], pH[CPML ? C : 1];
    R bE[CPML ? C : 1], aE[CPML ? C : 1], bH[CPML ? C : 1], aH[CPML ? C : 1];
    uint32_t eZone, hZone;         // bit i: node i has an E / H psi
};

// Whole-wave neighbour moves with DPP (gfx9 wave_shl:1 / wave_shr:1): lane i
// receives lane i+1's value (down) or lane i-1's (up); the lane with no source
// receives 0, written by the move itself (bound_ctrl), so no zeroed
// destination has to be set up first.  One v_mov_b32_dpp per 32-bit half, no
// LDS crossbar trip.
__device__ __forceinline__ int dpp_down1(int x)
{
    return __builtin_amdgcn_mov_dpp(x, 0x130, 0xF, 0xF, true);
}
__device__ __forceinline__ int dpp_up1(int x)
{
    return __builtin_amdgcn_mov_dpp(x, 0x138, 0xF, 0xF, true);
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

// The vector a lane moves C nodes of T with: 16 bytes, or the whole chunk
// where it is smaller (C = 2 in FP32).
template <int B>
struct VecOf;
template <>
struct VecOf<16> {
    typedef uint4 type;
};
template <>
struct VecOf<8> {
    typedef uint2 type;
};
template <typename T, int C>
struct ChunkVec {
    static constexpr int bytes = C * (int)sizeof(T) >= 16 ? 16 : C * (int)sizeof(T);
    static constexpr int per = bytes / (int)sizeof(T);
    typedef typename VecOf<bytes>::type type;
    static_assert(C % per == 0, "C must fill whole vectors");
};

// Load nodes [k0, k0+C) of array a (grid-local pointer); nodes >= lim read 0.
template <typename T, int C>
__device__ __forceinline__ void load_chunk(const T *a, int64_t k0, int64_t lim, T (&v)[C])
{
    typedef ChunkVec<T, C> CV;
    constexpr int per = CV::per;
    if (k0 >= 0 && k0 + C <= lim && (k0 % per) == 0) {
        const typename CV::type *p = reinterpret_cast<const typename CV::type *>(a + k0);
#pragma unroll
        for (int q = 0; q < C / per; ++q) {
            const typename CV::type u = p[q];
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
    typedef ChunkVec<T, C> CV;
    constexpr int per = CV::per;
    if (k0 >= lo && k0 + C <= hi && (k0 % per) == 0) {
        typename CV::type *p = reinterpret_cast<typename CV::type *>(a + k0);
#pragma unroll
        for (int q = 0; q < C / per; ++q) {
            typename CV::type u;
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

// load_chunk into registers of type R (widened from the storage type T).
template <typename T, int C, typename R>
__device__ __forceinline__ void load_chunk_as(const T *a, int64_t k0, int64_t lim, R (&v)[C])
{
    if constexpr (sizeof(T) == sizeof(R)) {
        load_chunk<T, C>(a, k0, lim, v);
    } else {
        T t[C];
        load_chunk<T, C>(a, k0, lim, t);
#pragma unroll
        for (int i = 0; i < C; ++i) v[i] = (R)t[i];
    }
}

// store_chunk from registers of type R (each value rounded once to T).
template <typename T, int C, typename R>
__device__ __forceinline__ void store_chunk_as(T *a, int64_t k0, int64_t lo, int64_t hi, const R (&v)[C])
{
    if constexpr (sizeof(T) == sizeof(R)) {
        store_chunk<T, C>(a, k0, lo, hi, v);
    } else {
        T t[C];
#pragma unroll
        for (int i = 0; i < C; ++i) t[i] = (T)v[i];
        store_chunk<T, C>(a, k0, lo, hi, t);
    }
}

// x, hidden from the optimiser.  A coefficient negated through here reaches
// the step's FMAs as a plain register, so they compile to the two-operand
// accumulate form; a visible negation is folded into the three-operand form
// as a source modifier, which issues at half the rate for FP32 on gfx950.
template <typename T>
__device__ __forceinline__ T opaque(T x)
{
    asm volatile("" : "+v"(x));
    return x;
}

// Load the lane's chunk starting at grid node k0 of grid b (buffer `buf`).
template <typename T, int C, bool PLASMA, bool CPML, bool JF = false>
__device__ __forceinline__ void chunk_load(Chunk<T, C, PLASMA, CPML, JF> &ck, const Grids &g,
                                           const State<T> &s, int buf, int b, int64_t off,
                                           int64_t n, int64_t k0, int64_t lim)
{
    typedef typename Chunk<T, C, PLASMA, CPML, JF>::R R;
    ck.nch = opaque<R>(-(R)g.ch);
    ck.nce = opaque<R>(-(R)g.ce);
    load_chunk_as<T, C>(s.E[buf] + off, k0, lim, ck.E);
    load_chunk_as<T, C>(s.H[buf] + off, k0, lim, ck.H);
    if constexpr (PLASMA && !JF && !CPML) {
        // the step coefficients from the table built at create (the values
        // node_coef_t gives, -CH already negated); padding and nodes past the
        // grid's end read zeros and are never stored.  (CPML tiles, which
        // also hold the psi registers, build theirs below: loading them
        // would raise the kernel's peak register count past the file.)
        load_chunk<double, C>(s.J[buf] + off, k0, lim, ck.J);
        const int64_t N = g.coef_n;
        double eP[C], nH[C], a[C], qc[C];
        load_chunk<double, C>(g.coef + off, k0, lim, eP);
        load_chunk<double, C>(g.coef + N + off, k0, lim, nH);
        load_chunk<double, C>(g.coef + 2 * N + off, k0, lim, a);
        load_chunk<double, C>(g.coef + 3 * N + off, k0, lim, qc);
#pragma unroll
        for (int i = 0; i < C; ++i) {
            ck.cf[i].eP = (R)eP[i];
            ck.cf[i].eH = (R)nH[i];
            ck.cf[i].a = a[i];
            ck.cf[i].qc = qc[i];
        }
    } else if constexpr (PLASMA) {
        // built here from wp2 and nu (CPML tiles; the ablation, which carries
        // J itself with FP32 coefficients)
        if constexpr (JF) {
            double Jd[C];
            load_chunk<double, C>(s.J[buf] + off, k0, lim, Jd);
#pragma unroll
            for (int i = 0; i < C; ++i) {
                ck.J[i] = (float)Jd[i];
                ck.Ed[i] = ck.E[i];
            }
        } else {
            load_chunk<double, C>(s.J[buf] + off, k0, lim, ck.J);
        }
        double w[C], v[C];
        load_chunk<double, C>(g.wp2 + off, k0, lim, w);
        load_chunk<double, C>(g.nu + off, k0, lim, v);
#pragma unroll
        for (int i = 0; i < C; ++i) {
            ck.cf[i] = node_coef_t<R>(w[i], v[i], g.dt, g.dz, g.scheme);
            if constexpr (JF) ck.cf[i].eJ = opaque<R>(-ck.cf[i].eJ);   // the Q carry needs no CJ
            ck.cf[i].eH = opaque<R>(-ck.cf[i].eH);
            if constexpr (JF) {
                ck.jc[3 * i] = (float)(ck.cf[i].a - 1.0);
                ck.jc[3 * i + 1] = (float)ck.cf[i].b1;
                ck.jc[3 * i + 2] = (float)ck.cf[i].b2;
            }
        }
    }
    if constexpr (CPML) {
        ck.eZone = ck.hZone = 0;
        const int P = g.cpmlP;
#pragma unroll
        for (int i = 0; i < C; ++i) {
            const int64_t k = k0 + i;
            ck.pE[i] = ck.pH[i] = (R)0;
            ck.bE[i] = ck.bH[i] = (R)1;
            ck.aE[i] = ck.aH[i] = (R)0;
            if (k < 0 || k >= lim) continue;   // k = -1: a tile shifted off node 0
            int slot = -1, tab = 0;
            // E psi: nodes 1..P-1 and n-P..n-2 (depth d -> table d-1)
            if (k >= 1 && k < P) { tab = P - 1 - (int)k; slot = (int)k; }
            else if (k > n - 1 - P && k <= n - 2) { tab = (int)(k - (n - 1 - P)) - 1; slot = P + (int)(k - (n - P)); }
            if (slot >= 0) {
                ck.eZone |= 1u << i;
                ck.pE[i] = (R)s.psiE[buf][(int64_t)b * 2 * P + slot];
                ck.bE[i] = (R)g.cpml[tab];
                ck.aE[i] = (R)g.cpml[P + tab];
            }
            slot = -1;
            // H psi: nodes 0..P-1 and n-1-P..n-2 (depth j+1/2 -> table j)
            if (k < P) { tab = P - 1 - (int)k; slot = (int)k; }
            else if (k >= n - 1 - P && k <= n - 2) { tab = (int)(k - (n - 1 - P)); slot = P + tab; }
            if (slot >= 0) {
                ck.hZone |= 1u << i;
                ck.pH[i] = (R)s.psiH[buf][(int64_t)b * 2 * P + slot];
                ck.bH[i] = (R)g.cpml[2 * P + tab];
                ck.aH[i] = (R)g.cpml[3 * P + tab];
            }
        }
    }
}

template <typename T, int C, bool PLASMA, bool CPML, bool JF = false>
__device__ __forceinline__ void chunk_store(const Chunk<T, C, PLASMA, CPML, JF> &ck, const Grids &g,
                                            const State<T> &s, int buf, int b, int64_t off,
                                            int64_t n, int64_t k0, int64_t lo, int64_t hi)
{
    store_chunk_as<T, C>(s.E[buf] + off, k0, lo, hi, ck.E);
    store_chunk_as<T, C>(s.H[buf] + off, k0, lo, hi < n ? hi : n - 1, ck.H);   // H has n-1 nodes
    if constexpr (PLASMA && JF) {
        double Jd[C];
#pragma unroll
        for (int i = 0; i < C; ++i) Jd[i] = (double)ck.J[i];
        store_chunk<double, C>(s.J[buf] + off, k0, lo, hi, Jd);
    } else if constexpr (PLASMA) {
        store_chunk<double, C>(s.J[buf] + off, k0, lo, hi, ck.J);
    }
    if constexpr (CPML) {
        const int P = g.cpmlP;
#pragma unroll
        for (int i = 0; i < C; ++i) {
            const int64_t k = k0 + i;
            if (k < lo || k >= hi) continue;
            if (ck.eZone & (1u << i)) {
                const int slot = (k < P) ? (int)k : P + (int)(k - (n - P));
                s.psiE[buf][(int64_t)b * 2 * P + slot] = (T)ck.pE[i];
            }
            if (ck.hZone & (1u << i)) {
                const int slot = (k < P) ? (int)k : P + (int)(k - (n - 1 - P));
                s.psiH[buf][(int64_t)b * 2 * P + slot] = (T)ck.pH[i];
            }
        }
    }
}

// H^{n+1/2} of the chunk; Er = E of the next node after the chunk.  (The
// update of h_update, with the coefficient held negated.)
template <typename T, int C, bool PLASMA, bool CPML, bool JF = false>
__device__ __forceinline__ void chunk_h(Chunk<T, C, PLASMA, CPML, JF> &ck,
                                        typename Chunk<T, C, PLASMA, CPML, JF>::R Er)
{
    typedef typename Chunk<T, C, PLASMA, CPML, JF>::R R;
#pragma unroll
    for (int i = 0; i < C; ++i) {
        const R er = (i + 1 < C) ? ck.E[i + 1] : Er;
        if constexpr (CPML) {
            if (ck.hZone & (1u << i)) {
                const R dE = er - ck.E[i];
                ck.pH[i] = fmat(ck.aH[i], dE, ck.bH[i] * ck.pH[i]);
                ck.H[i] = fmat(ck.nch, dE + ck.pH[i], ck.H[i]);
                continue;
            }
        }
        ck.H[i] = fmat(ck.nch, er - ck.E[i], ck.H[i]);
    }
}

// E^{n+1} (before the source) of the chunk; Hl = H of the node before the
// chunk.
template <typename T, int C, bool PLASMA, bool CPML, bool JF = false>
__device__ __forceinline__ void chunk_e(Chunk<T, C, PLASMA, CPML, JF> &ck,
                                        typename Chunk<T, C, PLASMA, CPML, JF>::R Hl)
{
    typedef typename Chunk<T, C, PLASMA, CPML, JF>::R R;
#pragma unroll
    for (int i = 0; i < C; ++i) {
        R curl = ck.H[i] - ((i > 0) ? ck.H[i - 1] : Hl);
        if constexpr (CPML) {
            if (ck.eZone & (1u << i)) {
                ck.pE[i] = fmat(ck.aE[i], curl, ck.bE[i] * ck.pE[i]);
                curl = curl + ck.pE[i];
            }
        }
        if constexpr (PLASMA && JF) {
            ck.E[i] = e_update_plasma_neg(ck.E[i], ck.J[i], curl, ck.cf[i].eJ, ck.cf[i].eH, ck.cf[i].eA);
        } else if constexpr (PLASMA) {
            // Q^n from E^n before E^n is overwritten, then E^{n+1} from Q^{n-1}
            // (e_update_plasma_q, q_update); the plasma formula reproduces the
            // vacuum update at vacuum nodes
            const double qn = q_update<R>(ck.J[i], (double)ck.E[i], ck.cf[i]);
            ck.E[i] = e_update_plasma_qneg(ck.E[i], ck.J[i], curl, ck.cf[i].eH, ck.cf[i].eP);
            ck.J[i] = qn;
        } else {
            ck.E[i] = fmat(ck.nce, curl, ck.E[i]);   // e_update_vac
        }
    }
}

// The ablation's J update (after the source), with E_old the copy of E^n kept
// from the previous step; at vacuum nodes a*0 + 0*E + 0*E keeps J at +0.  The
// Mur ends rewrite E after this and leave their copy stale, which is harmless:
// end nodes carry no plasma (b1 = 0).  (The carried Q is advanced inside
// chunk_e.)
template <typename T, int C, bool PLASMA, bool CPML, bool JF = false>
__device__ __forceinline__ void chunk_j(Chunk<T, C, PLASMA, CPML, JF> &ck)
{
    if constexpr (PLASMA && JF) {
        // the ablation: the operations of j_update_delta on the FP32 coefficients
#pragma unroll
        for (int i = 0; i < C; ++i) {
            const float en = ck.E[i];
            ck.J[i] = fmat(ck.jc[3 * i + 2], en, fmat(ck.jc[3 * i + 1], ck.Ed[i], fmat(ck.jc[3 * i], ck.J[i], ck.J[i])));
            ck.Ed[i] = en;
        }
    }
}

// One time step of a chunk that holds no grid end and no source: H, then E
// with the carried Q (or, in the ablation, E then J).
template <typename T, int C, bool PLASMA, bool CPML, bool JF, typename GetEr, typename GetHl>
__device__ __forceinline__ void chunk_step_plain(Chunk<T, C, PLASMA, CPML, JF> &ck, const Grids &g,
                                                 GetEr get_er, GetHl get_hl)
{
    chunk_h<T, C, PLASMA, CPML, JF>(ck, get_er(ck.E[0]));
    chunk_e<T, C, PLASMA, CPML, JF>(ck, get_hl(ck.H[C - 1]));
    chunk_j<T, C, PLASMA, CPML, JF>(ck);
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

// acc with lane l set to x (x and l wave-uniform; a select, bit for bit).
__device__ __forceinline__ double writelane_d(double acc, double x, int l, int lane)
{
    return lane == l ? x : acc;
}

// The end values the Mur updates read, E^n at nodes 0, 1 and n-1, n-2, held
// from one step to the next: each equals what the previous step wrote (the
// end node) or read (its neighbour, which later sub-steps of that step leave
// alone).  Meaningful only in the lane holding the end.
template <typename T>
struct EndCarry {
    T e0, e1, eR, eR1;
};

// E at node 1 in the lane holding node 0 (register left_reg of lane 0):
// register left_reg + 1 of the same lane, or, with two nodes a lane and node 0
// in register 1, the next lane's register 0.  Every lane takes part in the
// cross-lane move.
template <typename T, int C>
__device__ __forceinline__ T node1_of_left(const T (&E)[C], int left_reg)
{
    if constexpr (C > 2) {
        return left_reg ? E[2] : E[1];
    } else {
        const T nx = shfl_down1(E[0]);
        return left_reg ? nx : E[1];
    }
}

template <typename T, int C, bool FX = false>
__device__ __forceinline__ void ends_init(const T (&E)[C], const WaveRole &r, EndCarry<T> &c)
{
    if constexpr (FX) {
        // node 0 in register 0, node n-1 in register C-1 (see TILE_FIXED)
        c.e0 = E[0];
        c.e1 = E[1];
        c.eR = E[C - 1];
        c.eR1 = E[C - 2];
        return;
    }
    c.e0 = r.left_reg ? E[1] : E[0];
    c.e1 = node1_of_left<T, C>(E, r.left_reg);
    const int ir = r.right_reg;
    c.eR = upick<T, C>(E, ir);
    c.eR1 = ir ? upick<T, C>(E, ir - 1) : shfl_up1(E[C - 1]);
}

// One full time step of a wave holding a grid end, the source or a probe: H;
// E with the carried Q (the Q update reads E^n first); the source, added to
// E^{n+1} (eq.(15)); the ablation's J update; then the ends (first-order Mur,
// or PEC E = 0).  sv: the source value of this step.  Only the parts of the
// roles in mask RM are compiled in.
// Every part runs in every such wave, as selects whose lane condition is
// false where the wave does not hold the node: no branch, so the registers
// need no merging copies.
template <typename T, int C, bool PLASMA, bool CPML, int RM, bool JF, typename GetEr, typename GetHl>
__device__ __forceinline__ void chunk_step(Chunk<T, C, PLASMA, CPML, JF> &ck, const Grids &g,
                                           const WaveRole &r, int lane,
                                           EndCarry<typename Chunk<T, C, PLASMA, CPML, JF>::R> &c, double sv,
                                           GetEr get_er, GetHl get_hl)
{
    typedef typename Chunk<T, C, PLASMA, CPML, JF>::R R;
    constexpr bool FX = RM > 0 && (RM & kRoleFixed) != 0;
    chunk_h<T, C, PLASMA, CPML, JF>(ck, get_er(ck.E[0]));
    chunk_e<T, C, PLASMA, CPML, JF>(ck, get_hl(ck.H[C - 1]));
    if constexpr ((RM & kRoleSrc) != 0 && FX) {
        ck.E[0] = lane == r.src_lane ? add_source<R>(ck.E[0], sv) : ck.E[0];
    } else if constexpr ((RM & kRoleSrc) != 0) {
        uput<R, C>(ck.E, r.src_reg, lane == r.src_lane, add_source<R>(upick<R, C>(ck.E, r.src_reg), sv));
    }
    chunk_j<T, C, PLASMA, CPML, JF>(ck);
    const bool mur = g.bc == 0;
    if constexpr ((RM & kRoleLeft) != 0 && FX) {
        const R v = mur ? (R)(c.e1 + (R)g.cm * (ck.E[1] - c.e0)) : (R)0;
        c.e1 = ck.E[1];
        ck.E[0] = lane == r.left_lane ? v : ck.E[0];
        c.e0 = v;
    } else if constexpr ((RM & kRoleLeft) != 0) {
        const R en1 = node1_of_left<R, C>(ck.E, r.left_reg);
        const R v = mur ? (R)(c.e1 + (R)g.cm * (en1 - c.e0)) : (R)0;
        const bool here = lane == r.left_lane;
        ck.E[0] = (here && !r.left_reg) ? v : ck.E[0];
        ck.E[1] = (here && r.left_reg) ? v : ck.E[1];
        c.e0 = v;
        c.e1 = en1;
    }
    if constexpr ((RM & kRoleRight) != 0 && FX) {
        const R en1 = ck.E[C - 2];
        const R v = mur ? (R)(c.eR1 + (R)g.cm * (en1 - c.eR)) : (R)0;
        ck.E[C - 1] = lane == r.right_lane ? v : ck.E[C - 1];
        c.eR = v;
        c.eR1 = en1;
    } else if constexpr ((RM & kRoleRight) != 0) {
        const int ir = r.right_reg;
        const R prev = shfl_up1(ck.E[C - 1]);
        const R left1 = upick<R, C>(ck.E, ir > 0 ? ir - 1 : 0);
        const R en1 = ir > 0 ? left1 : prev;
        const R v = mur ? (R)(c.eR1 + (R)g.cm * (en1 - c.eR)) : (R)0;
        uput<R, C>(ck.E, ir, lane == r.right_lane, v);
        c.eR = v;
        c.eR1 = en1;
    }
}



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
// steps, one per lane of the window's table, broadcast from lane st.  The
// samples of up to two probes are gathered the other way round: step st's
// sample goes into lane st of a register, and the run ends with one
// coalesced store a probe, so the steps themselves issue no store and change
// no exec mask (a wave with more probes stores each sample as it is taken).
// (Every cross-lane read here takes a value all lanes computed: a value
// computed only in some lanes would be stale in the lane that is read.)
template <typename T, int C, bool PLASMA, bool CPML, int RM = kRoleAll, bool JF = false, typename GetEr,
          typename GetHl, typename Post>
__device__ __forceinline__ void run_role(Chunk<T, C, PLASMA, CPML, JF> &ck, const Grids &g, const WaveRole &r,
                                         const WaveProbes &wp, int lane, int b, int64_t wave_lo, int64_t plo,
                                         int64_t phi, int nsteps, int slot0, GetEr er, GetHl hl, Post post)
{
    constexpr bool SRC = (RM & kRoleSrc) != 0;
    constexpr bool FX = RM > 0 && (RM & kRoleFixed) != 0;
    typedef typename Chunk<T, C, PLASMA, CPML, JF>::R R;
    EndCarry<R> c;
    ends_init<R, C, FX>(ck.E, r, c);
    for (int base = 0; base < nsteps; base += 64) {
        const int cnt = nsteps - base < 64 ? nsteps - base : 64;
        const int slot = slot0 + base;
        double svl = 0.0;
        if (SRC && r.src_lane >= 0) {
            const int i = slot + lane;
            svl = g.srcv[i < g.SB ? i : g.SB - 1];
        }
        double pb0 = 0.0, pb1 = 0.0;   // the run's samples of probes 0 and 1, lane st: step st
        auto one = [&](int st) {
            const double sv = (SRC && r.src_lane >= 0) ? readlane_d(svl, st) : 0.0;
            chunk_step<T, C, PLASMA, CPML, RM, JF>(ck, g, r, lane, c, sv, er, hl);
            post(base + st);
            if constexpr ((RM & kRoleProbe) == 0) {
            } else if constexpr (FX) {
                // at most two probes, each in register 0 of its lane
                if (wp.n > 0) pb0 = writelane_d(pb0, readlane_d((double)ck.E[0], wp.lane[0]), st, lane);
                if (wp.n > 1) pb1 = writelane_d(pb1, readlane_d((double)ck.E[0], wp.lane[1]), st, lane);
            } else if (wp.n > 2) {
                wave_probes<R, C>(g, b, wave_lo, plo, phi, lane, ck.E, slot + st);
            } else {
                if (wp.n > 0)
                    pb0 = writelane_d(pb0, readlane_d((double)upick<R, C>(ck.E, wp.reg[0]), wp.lane[0]), st, lane);
                if (wp.n > 1)
                    pb1 = writelane_d(pb1, readlane_d((double)upick<R, C>(ck.E, wp.reg[1]), wp.lane[1]), st, lane);
            }
        };
        int st = 0;
        for (; st + 2 <= cnt; st += 2) {
            one(st);
            one(st + 1);
        }
        if (st < cnt) one(st);
        if constexpr ((RM & kRoleProbe) != 0) {
            if (FX || wp.n <= 2) {
                if (wp.n > 0 && lane < cnt) g.samp[wp.row[0] + slot + lane] = pb0;
                if (wp.n > 1 && lane < cnt) g.samp[wp.row[1] + slot + lane] = pb1;
            }
        }
    }
}

// run_role for a wave of a small mixed role class: the wave takes the code
// compiled for the first role group covering its roles (the groups of
// role_group), chosen at run time.  Used where a class is too small to be
// split into per-group launches (its launch is latency bound, so the
// registers the several instantiations hold do not cost occupancy).
template <typename T, int C, bool PLASMA, bool CPML, bool JF, typename GetEr, typename GetHl, typename Post>
__device__ __forceinline__ void run_role_any(Chunk<T, C, PLASMA, CPML, JF> &ck, const Grids &g, const WaveRole &r,
                                             const WaveProbes &wp, int lane, int b, int64_t wave_lo, int64_t plo,
                                             int64_t phi, int nsteps, int slot0, GetEr er, GetHl hl, Post post)
{
    const int rm = (r.src_lane >= 0 ? kRoleSrc : 0) | (r.left_lane >= 0 ? kRoleLeft : 0) |
                   (r.right_lane >= 0 ? kRoleRight : 0);
#define FDTDP_ROLE(M) \
    run_role<T, C, PLASMA, CPML, M>(ck, g, r, wp, lane, b, wave_lo, plo, phi, nsteps, slot0, er, hl, post)
    if constexpr (CPML) {
        // tiles of a CPML class carry the psi registers too.  At 512 nodes
        // and more: one variant (the full role step, whose parts are no-ops
        // where the wave lacks the node); with two or more those
        // instantiations spill.  At 256 nodes (short grids, where these
        // latency-bound tiles set the pass time) the two ends alone, the
        // usual CPML tiles of a grid longer than a few tiles, get their own.
        if constexpr (C <= 4) {
            switch (rm) {
            case kRoleLeft: FDTDP_ROLE(kRoleLeft | kRoleProbe); return;
            case kRoleRight: FDTDP_ROLE(kRoleRight | kRoleProbe); return;
            default: FDTDP_ROLE(kRoleAll); return;
            }
        } else {
            (void)rm;
            FDTDP_ROLE(kRoleAll);
            return;
        }
    }
    switch (rm) {
    case 0: FDTDP_ROLE(kRoleProbe); break;
    case kRoleSrc: FDTDP_ROLE(kRoleSrc | kRoleProbe); break;
    case kRoleLeft: FDTDP_ROLE(kRoleLeft | kRoleProbe); break;
    case kRoleRight: FDTDP_ROLE(kRoleRight | kRoleProbe); break;
    case kRoleLeft | kRoleSrc: FDTDP_ROLE(kRoleLeft | kRoleSrc | kRoleProbe); break;
    default: FDTDP_ROLE(kRoleAll); break;
    }
#undef FDTDP_ROLE
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


}  // namespace fdtdp
#endif
