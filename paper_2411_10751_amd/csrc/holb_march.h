// Plane-marching fused step for the thermal family (variants >= 1).
//
// The thermal-dissipation source needs grad theta of the same time step
// (central differences, Section 3.2), i.e. theta of the neighbours, which is
// a moment of *their* pulled populations.  Instead of a separate field pass,
// a workgroup owns a lateral tile (x, y in 3D; x in 2D) plus a one-cell ring
// and marches along the last axis: at each plane it pulls the populations of
// the tile and ring, writes theta into a 4-plane LDS ring, and collides the
// previous plane, whose theta neighbours (lateral and both march neighbours)
// are now all in LDS.  Every interior population is read once and written
// once per step; the ring adds (tile + ring) / tile extra reads, which mostly
// hit L2 because the neighbouring tile pulls the same cells at the same time.
// Wall planes (TMS, Section 4.3) are handled in the same pass.
#pragma once

#include "holb_cell.h"
#include "holb_internal.h"

namespace holb {

template <int TX_, int TY_, int NCH_>
struct MarchShape {
    static constexpr int TX = TX_, TY = TY_, NCH = NCH_;  // NCH: chunks along the march axis (0 = auto)
};

template <class L, int ST, class S>
__global__ void __launch_bounds__(S::TX* S::TY)
k_march(const KParams p, const typename Codec<ST>::T* __restrict__ fin, typename Codec<ST>::T* __restrict__ fout,
        const float* __restrict__ tgt_in, float* __restrict__ tgt_out, int ntx, int nty, int nch, int chunk)
{
    using LL = Lat<L>;
    constexpr bool D3 = L::D == 3;
    constexpr int TX = S::TX, TY = D3 ? S::TY : 1;
    constexpr int IX = TX - 2, IY = D3 ? TY - 2 : 1;
    __shared__ float th[4][TY][TX];  // theta - theta0 of four consecutive planes

    const int tx = threadIdx.x, ty = D3 ? threadIdx.y : 0;
    // XCD-aware order: each XCD gets a contiguous run of (tile, chunk) items.
    const int nb = gridDim.x;
    int b = blockIdx.x;
    if (nb % 8 == 0) b = (b % 8) * (nb / 8) + b / 8;
    const int tile_x = b % ntx;
    int r = b / ntx;
    const int tile_y = D3 ? r % nty : 0;
    const int ck = D3 ? r / nty : r;
    const int nm = D3 ? p.nz : p.ny;  // march extent
    const int z0 = ck * chunk, z1 = min(z0 + chunk, nm);

    const int gx = tile_x * IX - 1 + tx;            // unwrapped lateral coordinates
    const int gy = D3 ? tile_y * IY - 1 + ty : 0;
    const int x = wrapc(gx, p.nx);
    const int y = D3 ? wrapc(gy, p.ny) : 0;
    const bool interior = tx >= 1 && tx <= IX && gx < p.nx && (!D3 || (ty >= 1 && ty <= IY && gy < p.ny));

    const bool walls = p.walls;
    const int pstart = walls ? max(z0 - 1, 0) : z0 - 1;
    const int pend = walls ? min(z1, nm - 1) : z1;  // last plane pulled

    float cur[L::Q], nxt[L::Q];
#pragma unroll
    for (int i = 0; i < L::Q; ++i) cur[i] = 0.f;

    for (int pz = pstart; pz <= z1; ++pz) {
        // 1. pull plane pz, its theta into the LDS ring
        if (pz <= pend) {
            const int zz = walls ? pz : wrapc(pz, nm);
            float dr, j[3], ed;
            if (D3) load_state<L, ST>(p, fin, tgt_in, x, y, zz, nxt, dr, j, ed);
            else load_state<L, ST>(p, fin, tgt_in, x, zz, 0, nxt, dr, j, ed);
            const float z3[3] = {0.f, 0.f, 0.f};
            Macro mq;
            // flags are raised once, at the collision of the plane
            macro_from_moments<L, false>(p, dr, j, ed, z3, mq);
            th[pz & 3][ty][tx] = mq.dth;
        }
        __syncthreads();
        // 2. collide plane q = pz - 1
        const int q = pz - 1;
        if (q >= z0 && interior) {
            const int qq = walls ? q : wrapc(q, nm);
            float dr, j[3], ed;
            moments<L>(cur, dr, j, ed);
            const float z3[3] = {0.f, 0.f, 0.f};
            Macro m;
            macro_from_moments<L>(p, dr, j, ed, z3, m);
            float gT[3];
            gT[0] = 0.5f * (th[q & 3][ty][tx + 1] - th[q & 3][ty][tx - 1]);
            float gm;
            if (walls && q == 0) gm = th[1][ty][tx] - th[0][ty][tx];
            else if (walls && q == nm - 1) gm = th[q & 3][ty][tx] - th[(q - 1) & 3][ty][tx];
            else gm = 0.5f * (th[(q + 1) & 3][ty][tx] - th[(q - 1) & 3][ty][tx]);
            if (D3) {
                gT[1] = 0.5f * (th[q & 3][ty + 1][tx] - th[q & 3][ty - 1][tx]);
                gT[2] = gm;
            } else {
                gT[1] = gm;
                gT[2] = 0.0f;
            }
            if (walls) {
                if (D3) write_targets<L>(p, tgt_out, x, y, qq, m);
                else write_targets<L>(p, tgt_out, x, qq, 0, m);
            }
            collide<L>(p, cur, m, p.hfac * m.rho * m.theta, gT, 0.0f);
            const int cell = D3 ? (qq * p.ny + y) * p.nx + x : qq * p.nx + x;
#pragma unroll
            for (int i = 0; i < L::Q; ++i)
                fout[(long long)i * p.pitch + cell] = Codec<ST>::enc(cur[i], p.dref[i]);
        }
#pragma unroll
        for (int i = 0; i < L::Q; ++i) cur[i] = nxt[i];
    }
}

// Variant table.  3D: tiles of (TX-2) x (TY-2) interior cells; 2D: strips of
// TX-2 cells.  NCH chunks along the march axis (0: one chunk per 64 planes).
template <class L>
struct MarchVariants;

template <>
struct MarchVariants<D3Q39> {
    static constexpr int N = 4;
};
template <>
struct MarchVariants<D2Q37> {
    static constexpr int N = 3;
};

template <class L, int ST, class S>
inline hipError_t launch_march_shape(const LaunchCtx& c, int chunk_target)
{
    using T = typename Codec<ST>::T;
    constexpr bool D3 = L::D == 3;
    const KParams& p = c.kp;
    const int IX = S::TX - 2, IY = D3 ? S::TY - 2 : 1;
    const int ntx = (p.nx + IX - 1) / IX;
    const int nty = D3 ? (p.ny + IY - 1) / IY : 1;
    const int nm = D3 ? p.nz : p.ny;
    const int chunk = chunk_target < nm ? chunk_target : nm;
    const int nch = (nm + chunk - 1) / chunk;
    const dim3 block(S::TX, D3 ? S::TY : 1);
    hipLaunchKernelGGL((k_march<L, ST, S>), dim3(ntx * nty * nch), block, 0, c.stream, p, (const T*)c.pop_in,
                       (T*)c.pop_out, c.tgt_in, c.tgt_out, ntx, nty, nch, chunk);
    return hipGetLastError();
}

inline int march_num_variants(const LaunchCtx& c)
{
    if (c.family != FAM_THERMAL) return 0;
    return c.lattice == 1 ? MarchVariants<D3Q39>::N : MarchVariants<D2Q37>::N;
}

inline bool march_variant_supported(const LaunchCtx& c, int v)
{
    if (c.family != FAM_THERMAL || v < 1) return false;
    const int nm = c.lattice == 1 ? c.kp.nz : c.kp.ny;
    const int nlat = c.kp.nx;
    // a tile must not cover a periodic lateral axis more than once
    if (c.lattice == 1) return v <= MarchVariants<D3Q39>::N && nlat >= 2 && c.kp.ny >= 2 && nm >= 1;
    return v <= MarchVariants<D2Q37>::N && nlat >= 2 && nm >= 1;
}

template <class L, int ST, int FAM>
hipError_t march_step(const LaunchCtx& c)
{
    if (FAM != FAM_THERMAL || !march_variant_supported(c, c.variant)) return hipErrorNotSupported;
    if constexpr (L::D == 3) {
        switch (c.variant) {
        case 1: return launch_march_shape<L, ST, MarchShape<34, 18, 0>>(c, 64);
        case 2: return launch_march_shape<L, ST, MarchShape<34, 18, 0>>(c, 32);
        case 3: return launch_march_shape<L, ST, MarchShape<66, 10, 0>>(c, 64);
        case 4: return launch_march_shape<L, ST, MarchShape<18, 34, 0>>(c, 64);
        }
    } else {
        switch (c.variant) {
        case 1: return launch_march_shape<L, ST, MarchShape<258, 1, 0>>(c, 32);
        case 2: return launch_march_shape<L, ST, MarchShape<130, 1, 0>>(c, 32);
        case 3: return launch_march_shape<L, ST, MarchShape<130, 1, 0>>(c, 64);
        }
    }
    return hipErrorNotSupported;
}

}  // namespace holb
