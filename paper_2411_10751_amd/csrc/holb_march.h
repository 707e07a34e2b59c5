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
// In a walled domain the layers that need the TMS closure (Section 4.3) are
// left to the generic kernels and the march covers the planes between them.
#pragma once

#include <stdio.h>

#include "holb_cell.h"
#include "holb_internal.h"

namespace holb {

template <int TX_, int TY_, int NCH_>
struct MarchShape {
    static constexpr int TX = TX_, TY = TY_, NCH = NCH_;  // NCH: chunks along the march axis (0 = auto)
};

// Work item of a marching workgroup: lateral tile and chunk of planes.
struct MarchItem {
    int x, y;        // wrapped lateral coordinates of this thread's column
    int z0, z1;      // planes [z0, z1) collided by the workgroup
    bool interior;   // column inside the tile (not the one-cell ring)
};

template <class L, class S>
__device__ __forceinline__ MarchItem march_item(const KParams& p, int ntx, int nty, int mlo, int chunk, int mhi)
{
    constexpr bool D3 = L::D == 3;
    constexpr int TX = S::TX, TY = D3 ? S::TY : 1;
    constexpr int IX = TX - 2, IY = D3 ? TY - 2 : 1;
    (void)TY;
    const int tx = threadIdx.x, ty = D3 ? threadIdx.y : 0;
    // XCD-aware order: each XCD gets a contiguous run of (tile, chunk) items.
    const int nb = gridDim.x;
    int b = blockIdx.x;
    if (nb % 8 == 0) b = (b % 8) * (nb / 8) + b / 8;
    const int tile_x = b % ntx;
    const int r = b / ntx;
    const int tile_y = D3 ? r % nty : 0;
    const int ck = D3 ? r / nty : r;
    MarchItem it;
    it.z0 = mlo + ck * chunk;
    it.z1 = min(it.z0 + chunk, mhi);
    const int gx = tile_x * IX - 1 + tx;  // unwrapped lateral coordinates
    const int gy = D3 ? tile_y * IY - 1 + ty : 0;
    it.x = wrapc(gx, p.nx);
    it.y = D3 ? wrapc(gy, p.ny) : 0;
    it.interior = tx >= 1 && tx <= IX && gx < p.nx && (!D3 || (ty >= 1 && ty <= IY && gy < p.ny));
    return it;
}

// theta - theta0 of plane pz into the LDS ring: pulled and reduced to moments,
// or, for the planes next to the marched range of a walled domain (which need
// the TMS closure), read from the field the wall pass wrote.
template <class L, int ST>
__device__ __forceinline__ float march_theta(const KParams& p, const typename Codec<ST>::T* __restrict__ fin,
                                             const float* __restrict__ aux_f, int x, int y, int pz, int mlo,
                                             int mhi, int nm, float (&f)[L::Q], Frame& fo)
{
    constexpr bool D3 = L::D == 3;
    if (p.walls && (pz < mlo || pz >= mhi))
        return aux_f[D3 ? ((long long)pz * p.ny + y) * p.nx + x : (long long)pz * p.nx + x];
    const int zz = wrapc(pz, nm);
    float dr, j[3], ed;
    if (D3) load_state<L, ST, false>(p, fin, nullptr, x, y, zz, f, fo, dr, j, ed);
    else load_state<L, ST, false>(p, fin, nullptr, x, zz, 0, f, fo, dr, j, ed);
    const float z3[3] = {0.f, 0.f, 0.f};
    Macro mq;
    // flags are raised once, at the collision of the plane
    macro_from_moments<L, false>(p, fo, dr, j, ed, z3, mq);
    return theta_field(p, fo, mq);
}

// Collision of plane q of the column from its pulled populations f (in frame
// fo) and the theta ring; writes the post-collision populations.
template <class L, int ST, int TY, int TX>
__device__ __forceinline__ void march_collide(const KParams& p, typename Codec<ST>::T* __restrict__ fout,
                                              const float (&th)[4][TY][TX], int tx, int ty, int x, int y, int q,
                                              int nm, float (&f)[L::Q], const Frame& fo)
{
    constexpr bool D3 = L::D == 3;
    const int qq = wrapc(q, nm);
    float dr, j[3], ed;
    moments<L>(f, dr, j, ed);
    const float z3[3] = {0.f, 0.f, 0.f};
    Macro m;
    macro_from_moments<L>(p, fo, dr, j, ed, z3, m);
    float gT[3];
    gT[0] = 0.5f * (th[q & 3][ty][tx + 1] - th[q & 3][ty][tx - 1]);
    const float gm = 0.5f * (th[(q + 1) & 3][ty][tx] - th[(q - 1) & 3][ty][tx]);
    if (D3) {
        gT[1] = 0.5f * (th[q & 3][ty + 1][tx] - th[q & 3][ty - 1][tx]);
        gT[2] = gm;
    } else {
        gT[1] = gm;
        gT[2] = 0.0f;
    }
    collide<L>(p, fo, f, m, p.hfac * m.rho * m.theta, gT, 0.0f);
    const long long cell = D3 ? ((long long)qq * p.ny + y) * p.nx + x : (long long)qq * p.nx + x;
    store_cell<L, ST>(p, fout, cell, f, fo, m.rho, m.thb);
}

// Planes [mlo, mhi) are collided; mlo = 0, mhi = nm for a periodic domain.
// In a walled domain the range excludes the three layers next to each wall,
// so no pull here needs the TMS closure.
template <class L, int ST, class S>
__global__ void __launch_bounds__(S::TX* S::TY)
k_march(const KParams p, const typename Codec<ST>::T* __restrict__ fin, typename Codec<ST>::T* __restrict__ fout,
        const float* __restrict__ aux_f, int ntx, int nty, int mlo, int mhi, int chunk)
{
    constexpr bool D3 = L::D == 3;
    constexpr int TX = S::TX, TY = D3 ? S::TY : 1;
    __shared__ float th[4][TY][TX];  // theta - theta0 of four consecutive planes

    const int tx = threadIdx.x, ty = D3 ? threadIdx.y : 0;
    const int nm = D3 ? p.nz : p.ny;  // march extent
    const MarchItem it = march_item<L, S>(p, ntx, nty, mlo, chunk, mhi);

    float cur[L::Q], nxt[L::Q];
    Frame fcur = {0.f, 0.f}, fnxt = {0.f, 0.f};
#pragma unroll
    for (int i = 0; i < L::Q; ++i) cur[i] = nxt[i] = 0.f;

    for (int pz = it.z0 - 1; pz <= it.z1; ++pz) {
        // 1. pull plane pz, its theta into the LDS ring
        th[pz & 3][ty][tx] = march_theta<L, ST>(p, fin, aux_f, it.x, it.y, pz, mlo, mhi, nm, nxt, fnxt);
        __syncthreads();
        // 2. collide plane q = pz - 1, pulled at the previous iteration
        const int q = pz - 1;
        if (q >= it.z0 && it.interior)
            march_collide<L, ST, TY, TX>(p, fout, th, tx, ty, it.x, it.y, q, nm, cur, fcur);
#pragma unroll
        for (int i = 0; i < L::Q; ++i) cur[i] = nxt[i];
        fcur = fnxt;
    }
}

// Low-register form: each plane is pulled twice -- once for its theta (the
// populations are reduced to moments at once), and again one plane later,
// when it is collided.  The second read follows the first by one plane of the
// tile, so it is served by L2 or the last-level cache rather than HBM, and
// only one set of populations is live, which leaves room for more waves per
// compute unit to hide the latency of the per-plane barrier.
template <class L, int ST, class S>
__global__ void __launch_bounds__(S::TX* S::TY)
k_march2(const KParams p, const typename Codec<ST>::T* __restrict__ fin, typename Codec<ST>::T* __restrict__ fout,
         const float* __restrict__ aux_f, int ntx, int nty, int mlo, int mhi, int chunk)
{
    constexpr bool D3 = L::D == 3;
    constexpr int TX = S::TX, TY = D3 ? S::TY : 1;
    __shared__ float th[4][TY][TX];

    const int tx = threadIdx.x, ty = D3 ? threadIdx.y : 0;
    const int nm = D3 ? p.nz : p.ny;
    const MarchItem it = march_item<L, S>(p, ntx, nty, mlo, chunk, mhi);

    for (int pz = it.z0 - 1; pz <= it.z1; ++pz) {
        {
            float f[L::Q];
            Frame fo;
            th[pz & 3][ty][tx] = march_theta<L, ST>(p, fin, aux_f, it.x, it.y, pz, mlo, mhi, nm, f, fo);
        }
        __syncthreads();
        const int q = pz - 1;
        if (q >= it.z0 && it.interior) {
            const int qq = wrapc(q, nm);
            float f[L::Q], dr, j[3], ed;
            Frame fo;
            if (D3) load_state<L, ST, false>(p, fin, nullptr, it.x, it.y, qq, f, fo, dr, j, ed);
            else load_state<L, ST, false>(p, fin, nullptr, it.x, qq, 0, f, fo, dr, j, ed);
            march_collide<L, ST, TY, TX>(p, fout, th, tx, ty, it.x, it.y, q, nm, f, fo);
        }
    }
}

// Variant table.  3D: tiles of (TX-2) x (TY-2) interior cells; 2D: strips of
// TX-2 cells.  NCH chunks along the march axis (0: one chunk per 64 planes).
template <class L>
struct MarchVariants;

template <>
struct MarchVariants<D3Q39> {
    static constexpr int N = 8;
};
template <>
struct MarchVariants<D2Q37> {
    static constexpr int N = 6;
};

template <class L, int ST, class S, bool TWICE = false>
inline hipError_t launch_march_shape(const LaunchCtx& c, int chunk_target, int mlo, int mhi)
{
    using T = typename Codec<ST>::T;
    constexpr bool D3 = L::D == 3;
    const KParams& p = c.kp;
    const int IX = S::TX - 2, IY = D3 ? S::TY - 2 : 1;
    const int ntx = (p.nx + IX - 1) / IX;
    const int nty = D3 ? (p.ny + IY - 1) / IY : 1;
    const int nmarch = mhi - mlo;
    if (nmarch <= 0) return hipSuccess;
    const int chunk = chunk_target < nmarch ? chunk_target : nmarch;
    const int nch = (nmarch + chunk - 1) / chunk;
    const dim3 block(S::TX, D3 ? S::TY : 1);
    if (TWICE)
        hipLaunchKernelGGL((k_march2<L, ST, S>), dim3(ntx * nty * nch), block, 0, c.stream, p, (const T*)c.pop_in,
                           (T*)c.pop_out, c.aux_f, ntx, nty, mlo, mhi, chunk);
    else
        hipLaunchKernelGGL((k_march<L, ST, S>), dim3(ntx * nty * nch), block, 0, c.stream, p, (const T*)c.pop_in,
                           (T*)c.pop_out, c.aux_f, ntx, nty, mlo, mhi, chunk);
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

// Kernel name of a variant, as a profiler lists it without namespace and
// spaces (shapes as in march_step).
template <class L>
inline void march_kernel_name(int v, const char* lat, int st, char* name, size_t len)
{
    static const int s3[9][3] = {{0, 0, 0}, {34, 18, 0}, {34, 18, 0}, {66, 10, 0}, {18, 34, 0},
                                 {34, 18, 1}, {66, 10, 1}, {34, 10, 1}, {66, 6, 1}};
    static const int s2[7][2] = {{0, 0}, {258, 0}, {130, 0}, {130, 0}, {258, 1}, {130, 1}, {66, 1}};
    int tx, ty, twice;
    if (L::D == 3) { tx = s3[v][0]; ty = s3[v][1]; twice = s3[v][2]; }
    else { tx = s2[v][0]; ty = 1; twice = s2[v][1]; }
    snprintf(name, len, "%s<%s,%d,MarchShape<%d,%d,0>>", twice ? "k_march2" : "k_march", lat, st, tx, ty);
}

// Collide planes [mlo, mhi) along the last axis with the marching kernel of
// the context's variant.
template <class L, int ST, int FAM>
hipError_t march_step(const LaunchCtx& c, int mlo, int mhi)
{
    if (FAM != FAM_THERMAL || !march_variant_supported(c, c.variant)) return hipErrorNotSupported;
    if constexpr (L::D == 3) {
        switch (c.variant) {
        case 1: return launch_march_shape<L, ST, MarchShape<34, 18, 0>>(c, 64, mlo, mhi);
        case 2: return launch_march_shape<L, ST, MarchShape<34, 18, 0>>(c, 32, mlo, mhi);
        case 3: return launch_march_shape<L, ST, MarchShape<66, 10, 0>>(c, 64, mlo, mhi);
        case 4: return launch_march_shape<L, ST, MarchShape<18, 34, 0>>(c, 64, mlo, mhi);
        case 5: return launch_march_shape<L, ST, MarchShape<34, 18, 0>, true>(c, 64, mlo, mhi);
        case 6: return launch_march_shape<L, ST, MarchShape<66, 10, 0>, true>(c, 64, mlo, mhi);
        case 7: return launch_march_shape<L, ST, MarchShape<34, 10, 0>, true>(c, 64, mlo, mhi);
        case 8: return launch_march_shape<L, ST, MarchShape<66, 6, 0>, true>(c, 64, mlo, mhi);
        }
    } else {
        switch (c.variant) {
        case 1: return launch_march_shape<L, ST, MarchShape<258, 1, 0>>(c, 32, mlo, mhi);
        case 2: return launch_march_shape<L, ST, MarchShape<130, 1, 0>>(c, 32, mlo, mhi);
        case 3: return launch_march_shape<L, ST, MarchShape<130, 1, 0>>(c, 64, mlo, mhi);
        case 4: return launch_march_shape<L, ST, MarchShape<258, 1, 0>, true>(c, 32, mlo, mhi);
        case 5: return launch_march_shape<L, ST, MarchShape<130, 1, 0>, true>(c, 32, mlo, mhi);
        case 6: return launch_march_shape<L, ST, MarchShape<66, 1, 0>, true>(c, 64, mlo, mhi);
        }
    }
    return hipErrorNotSupported;
}

}  // namespace holb
