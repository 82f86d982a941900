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

#include "tile1d.h"

namespace fdtdp {

template <typename T, int C, int KLASS, bool ROLES, bool JF = false, int RM = kRoleAll>
__global__ __launch_bounds__(256) void k_tiled(Grids g, State<T> s, int cur, const Tile *tiles,
                                               int64_t ntiles, int nsteps, int slot0)
{
    // class 0: vacuum tiles; 1: tiles with plasma; 2: tiles touching a CPML
    // layer (which may also hold plasma further in).  ROLES: the tiles hold a
    // grid end, the source or a probe (a separate instantiation, so that the
    // bulk tiles' register budget is that of the plain step alone), at most
    // the roles of mask RM.  JF: the FP32 ablation of eq.(11)
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
    Chunk<T, C, PLASMA, CPML, JF> ck;
    typedef typename Chunk<T, C, PLASMA, CPML, JF>::R R;
    chunk_load<T, C, PLASMA, CPML>(ck, g, s, cur, b, off, n, k0, tl.hi);
    auto er = [](R e0) { return shfl_down1(e0); };
    auto hl = [](R h) { return shfl_up1(h); };
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
        if constexpr (RM < 0)   // a small mixed class: each wave picks its role code
            run_role_any<T, C, PLASMA, CPML>(ck, g, role, wp, lane, b, tl.lo, tl.out_lo, tl.out_hi, nsteps, slot0,
                                             er, hl, [](int) {});
        else
            run_role<T, C, PLASMA, CPML, RM>(ck, g, role, wp, lane, b, tl.lo, tl.out_lo, tl.out_hi, nsteps, slot0,
                                             er, hl, [](int) {});
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
    typedef typename Chunk<T, C, PLASMA, CPML>::R R;
    __shared__ R ldsE[WAVES];
    __shared__ R ldsH[WAVES];
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
    auto er = [&](R e0) {
        if (lane == 0) ldsE[w] = e0;
        __syncthreads();
        R v = shfl_down1(e0);
        if (lane == 63) v = (w + 1 < WAVES) ? ldsE[w + 1] : (R)0;
        return v;
    };
    auto hl = [&](R h) {
        if (lane == 63) ldsH[w] = h;
        __syncthreads();
        R v = shfl_up1(h);
        if (lane == 0) v = (w > 0) ? ldsH[w - 1] : (R)0;
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

// The FP32 delta-form ablation (g.jdelta): every class with the field
// updates in FP32 registers and, where there is plasma, J and eq.(11) in
// FP32, for 256- and 512-node tiles (the host refuses other shapes for it).
template <typename T, int C>
bool launch_tiled_jf(const Grids &g, State<T> &s, int cur, const Tile *tiles, int64_t ntiles, int klass,
                     int nsteps, int slot0, hipStream_t st)
{
    if constexpr (sizeof(T) == 4 && (C == 4 || C == 8)) {
        const unsigned nb = (unsigned)((ntiles + 3) / 4);
        if (klass == 0)
            hipLaunchKernelGGL((k_tiled<T, C, 0, false, true>), dim3(nb), dim3(256), 0, st, g, s, cur, tiles,
                               ntiles, nsteps, slot0);
        else if (klass == 1)
            hipLaunchKernelGGL((k_tiled<T, C, 1, false, true>), dim3(nb), dim3(256), 0, st, g, s, cur, tiles,
                               ntiles, nsteps, slot0);
        else if (klass == 2)
            hipLaunchKernelGGL((k_tiled<T, C, 2, true, true>), dim3(nb), dim3(256), 0, st, g, s, cur, tiles,
                               ntiles, nsteps, slot0);
        else
            hipLaunchKernelGGL((k_tiled<T, C, 1, true, true>), dim3(nb), dim3(256), 0, st, g, s, cur, tiles,
                               ntiles, nsteps, slot0);
        return true;
    }
    return false;
}

template <typename T, int C, int KLASS, int RM>
void launch_roles(const Grids &g, State<T> &s, int cur, const Tile *tiles, int64_t ntiles, int nsteps,
                  int slot0, hipStream_t st)
{
    const unsigned nb = (unsigned)((ntiles + 3) / 4);
    hipLaunchKernelGGL((k_tiled<T, C, KLASS, true, false, RM>), dim3(nb), dim3(256), 0, st, g, s, cur, tiles,
                       ntiles, nsteps, slot0);
}

// A role group's tiles with the step compiled for its roles (256- and
// 512-node tiles; wider tiles take the full step).
template <typename T, int C, int KLASS>
void launch_group(const Grids &g, State<T> &s, int cur, const Tile *tiles, int64_t ntiles, int group,
                  int nsteps, int slot0, hipStream_t st)
{
    if constexpr (C == 4 || C == 8) {
        switch (group) {
        case 0: return launch_roles<T, C, KLASS, kRoleProbe>(g, s, cur, tiles, ntiles, nsteps, slot0, st);
        case 1:
            return launch_roles<T, C, KLASS, kRoleSrc | kRoleProbe>(g, s, cur, tiles, ntiles, nsteps, slot0, st);
        case 2:
            return launch_roles<T, C, KLASS, kRoleLeft | kRoleProbe>(g, s, cur, tiles, ntiles, nsteps, slot0, st);
        case 3:
            return launch_roles<T, C, KLASS, kRoleRight | kRoleProbe>(g, s, cur, tiles, ntiles, nsteps, slot0,
                                                                     st);
        case 4:
            return launch_roles<T, C, KLASS, kRoleLeft | kRoleSrc | kRoleProbe>(g, s, cur, tiles, ntiles, nsteps,
                                                                               slot0, st);
        case -1: return launch_roles<T, C, KLASS, -1>(g, s, cur, tiles, ntiles, nsteps, slot0, st);
        default: break;
        }
        if constexpr (KLASS == 1) {
            // the fixed-register role step (TILE_FIXED tiles; role tiles only)
            constexpr int F = kRoleFixed | kRoleProbe;
            switch (group) {
            case 5: return launch_roles<T, C, KLASS, F>(g, s, cur, tiles, ntiles, nsteps, slot0, st);
            case 6: return launch_roles<T, C, KLASS, F | kRoleSrc>(g, s, cur, tiles, ntiles, nsteps, slot0, st);
            case 7: return launch_roles<T, C, KLASS, F | kRoleLeft>(g, s, cur, tiles, ntiles, nsteps, slot0, st);
            case 8: return launch_roles<T, C, KLASS, F | kRoleRight>(g, s, cur, tiles, ntiles, nsteps, slot0, st);
            case 9:
                return launch_roles<T, C, KLASS, F | kRoleLeft | kRoleSrc>(g, s, cur, tiles, ntiles, nsteps, slot0,
                                                                           st);
            default: break;
            }
        }
    }
    launch_roles<T, C, KLASS, kRoleAll>(g, s, cur, tiles, ntiles, nsteps, slot0, st);
}

template <typename T, int C>
void launch_tiled_c(const Grids &g, State<T> &s, int cur, const Tile *tiles, int64_t ntiles,
                    int klass, int nsteps, int slot0, hipStream_t st, int group)
{
    const unsigned nb = (unsigned)((ntiles + 3) / 4);
    if (g.jdelta && launch_tiled_jf<T, C>(g, s, cur, tiles, ntiles, klass, nsteps, slot0, st))
        return;
    if (klass == 0)
        hipLaunchKernelGGL((k_tiled<T, C, 0, false>), dim3(nb), dim3(256), 0, st, g, s, cur, tiles, ntiles,
                           nsteps, slot0);
    else if (klass == 1)
        hipLaunchKernelGGL((k_tiled<T, C, 1, false>), dim3(nb), dim3(256), 0, st, g, s, cur, tiles, ntiles,
                           nsteps, slot0);
    else if (klass == 2)
        launch_group<T, C, 2>(g, s, cur, tiles, ntiles, group, nsteps, slot0, st);
    else   // role tiles, vacuum or plasma: the plasma step reproduces the vacuum one
        launch_group<T, C, 1>(g, s, cur, tiles, ntiles, group, nsteps, slot0, st);
}

// Wide vacuum tiles (class 0 with a vacuum tile width of 1536 or 2048 nodes):
// the vacuum step only, the other classes are never this wide.
template <typename T, int C>
void launch_vacuum_c(const Grids &g, State<T> &s, int cur, const Tile *tiles, int64_t ntiles, int nsteps,
                     int slot0, hipStream_t st)
{
    const unsigned nb = (unsigned)((ntiles + 3) / 4);
    hipLaunchKernelGGL((k_tiled<T, C, 0, false>), dim3(nb), dim3(256), 0, st, g, s, cur, tiles, ntiles, nsteps,
                       slot0);
}

template <typename T>
void launch_tiled(const Grids &g, State<T> &s, int cur, const Tile *tiles, int64_t ntiles, int klass,
                  int C, int nsteps, int slot0, hipStream_t st, int waves, int group)
{
    if (waves == 2) return launch_tiledw_w<T, 2>(g, s, cur, tiles, ntiles, klass, C, nsteps, slot0, st);
    if (waves == 4) return launch_tiledw_w<T, 4>(g, s, cur, tiles, ntiles, klass, C, nsteps, slot0, st);
    if (waves == 8) return launch_tiledw_w<T, 8>(g, s, cur, tiles, ntiles, klass, C, nsteps, slot0, st);
    switch (C) {
    case 4: launch_tiled_c<T, 4>(g, s, cur, tiles, ntiles, klass, nsteps, slot0, st, group); break;
    case 8: launch_tiled_c<T, 8>(g, s, cur, tiles, ntiles, klass, nsteps, slot0, st, group); break;
    case 12: launch_tiled_c<T, 12>(g, s, cur, tiles, ntiles, klass, nsteps, slot0, st, group); break;
    case 24:
        if (klass == 0) launch_vacuum_c<T, 24>(g, s, cur, tiles, ntiles, nsteps, slot0, st);
        break;
    case 32:
        if (klass == 0) launch_vacuum_c<T, 32>(g, s, cur, tiles, ntiles, nsteps, slot0, st);
        break;
    default: launch_tiled_c<T, 16>(g, s, cur, tiles, ntiles, klass, nsteps, slot0, st, group); break;
    }
}

template void launch_tiled<float>(const Grids &, State<float> &, int, const Tile *, int64_t, int, int,
                                  int, int, hipStream_t, int, int);
template void launch_tiled<double>(const Grids &, State<double> &, int, const Tile *, int64_t, int,
                                   int, int, int, hipStream_t, int, int);

// ------------------------------------------------------------- resident

// One workgroup per bin of grids; slots[bin*WAVES + w] says which grid wave w
// holds.  Edge values cross waves through LDS: two barriers per step, taken by
// every wave of the workgroup (idle waves included) so the count matches.
template <typename T, int C, int WAVES>
__global__ __launch_bounds__(WAVES * 64) void k_resident(Grids g, State<T> s, int cur, int out,
                                                         const ResidentSlot *slots, int nsteps,
                                                         int slot0)
{
    typedef typename Chunk<T, C, true, false>::R R;
    __shared__ R ldsE[WAVES];
    __shared__ R ldsH[WAVES];
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
            ck.E[i] = ck.H[i] = (R)0;
            ck.J[i] = 0.0;
        }
    }
    const WaveRole role = active ? wave_role<C>(g, b, n, wave_lo, wave_hi) : WaveRole{-1, 0, -1, 0, -1, 1};
    auto get_er = [&](R e0) {
        if (lane == 0) ldsE[w] = e0;
        __syncthreads();
        R v = shfl_down1(e0);
        if (lane == 63) v = has_next ? ldsE[w + 1] : (R)0;
        return v;
    };
    auto get_hl = [&](R hl) {
        if (lane == 63) ldsH[w] = hl;
        __syncthreads();
        R v = shfl_up1(hl);
        if (lane == 0) v = has_prev ? ldsH[w - 1] : (R)0;
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
