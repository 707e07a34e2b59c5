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
// (On MI355X the split form -- a temperature pass, then the collision -- is
// faster at 256^3: the march needs about 250 registers for two decoded planes
// plus the loads in flight, i.e. two waves per SIMD, and loses a quarter of
// its lanes to the ring during the collision; the tuner picks per grid.)
// In a walled domain the layers that need the TMS closure (Section 4.3) are
// left to the generic kernels and the march covers the planes between them.
#pragma once

#include <stdio.h>

#include "holb_cell.h"
#include "holb_internal.h"

namespace holb {

// Lateral tile TX x TY (interior plus a one-cell ring) and the minimum number
// of waves per SIMD the compiler must allow (bounds the registers).
template <int TX_, int TY_, int WPE_>
struct MarchShape {
    static constexpr int TX = TX_, TY = TY_, WPE = WPE_;
};

// Work item of a marching workgroup: lateral tile and chunk of planes.
struct MarchItem {
    int x, y;        // wrapped lateral coordinates of this thread's column
    int z0, z1;      // planes [z0, z1) collided by the workgroup
    bool interior;   // column inside the tile (not the one-cell ring)
    int ox, oy;      // unwrapped lateral coordinates of thread (0, 0)
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
    it.ox = tile_x * IX - 1;
    it.oy = D3 ? tile_y * IY - 1 : 0;
    const int gx = it.ox + tx;  // unwrapped lateral coordinates
    const int gy = it.oy + (D3 ? ty : 0);
    it.x = wrapc(gx, p.nx);
    it.y = D3 ? wrapc(gy, p.ny) : 0;
    it.interior = tx >= 1 && tx <= IX && gx < p.nx && (!D3 || (ty >= 1 && ty <= IY && gy < p.ny));
    return it;
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

// Workgroup barrier for LDS exchange only: waits for this wave's LDS
// operations, not for its global loads, so that loads issued before the
// barrier stay in flight across it (__syncthreads() also fences global
// memory, which drains them).  The memory clobber keeps the compiler from
// moving memory accesses across it.
__device__ __forceinline__ void lds_barrier()
{
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// Software-pipelined march.  Per plane pz, each thread of the tile (interior
// and ring): decodes the populations of plane pz pulled during the previous
// plane, puts its theta into the LDS ring, and -- after a barrier -- issues
// the loads of plane pz + 1 before colliding plane pz - 1, so that the loads
// are in flight during the collision.  The frames of the seven planes a pull
// reaches are kept in an LDS ring of the tile plus a three-cell halo, so a
// population load is the only per-population global access.  Interior
// columns keep two decoded planes (pz - 1 for the collision, pz for the next
// one) and the raw loads of pz + 1.
template <class L, int ST, class S, bool PREFETCH>
__global__ void __launch_bounds__(S::TX* S::TY) __attribute__((amdgpu_waves_per_eu(S::WPE > 0 ? S::WPE : 1)))
k_march3(const KParams p, const typename Codec<ST>::T* __restrict__ fin, typename Codec<ST>::T* __restrict__ fout,
         const float* __restrict__ aux_f, int ntx, int nty, int mlo, int mhi, int chunk)
{
    using T = typename Codec<ST>::T;
    using LL = Lat<L>;
    constexpr bool D3 = L::D == 3;
    constexpr int TX = S::TX, TY = D3 ? S::TY : 1;
    constexpr int EX = TX + 6, EY = D3 ? TY + 6 : 1;
    constexpr int NT = TX * TY, NE = EX * EY;
    constexpr int FPT = (NE + NT - 1) / NT;  // frame words loaded per thread and plane
    __shared__ float th[4][TY][TX];
    __shared__ uint32_t frs[7][EY][EX];

    const int tx = threadIdx.x, ty = D3 ? threadIdx.y : 0, tid = ty * TX + tx;
    const int nm = D3 ? p.nz : p.ny;
    const MarchItem it = march_item<L, S>(p, ntx, nty, mlo, chunk, mhi);
    const uint32_t* __restrict__ fp = frame_plane<ST>(fin, p.pitch, L::Q);

    auto slot7 = [](int z) { return ((z % 7) + 7) % 7; };
    auto fetch_frames = [&](int zf, uint32_t (&w)[FPT]) {
        const int zz = wrapc(zf, nm);
#pragma unroll
        for (int k = 0; k < FPT; ++k) {
            const int e = tid + k * NT;
            w[k] = 0u;
            if (e < NE) {
                const int ex = e % EX, ey = e / EX;
                const int gx = wrapc(it.ox - 3 + ex, p.nx);
                const int cell = D3 ? (zz * p.ny + wrapc(it.oy - 3 + ey, p.ny)) * p.nx + gx : zz * p.nx + gx;
                w[k] = fp[cell];
            }
        }
    };
    auto store_frames = [&](int zf, const uint32_t (&w)[FPT]) {
        uint32_t* dst = &frs[slot7(zf)][0][0];
#pragma unroll
        for (int k = 0; k < FPT; ++k) {
            const int e = tid + k * NT;
            if (e < NE) dst[e] = w[k];
        }
    };
    const bool edge_plane_lo = p.walls != 0;  // planes outside [mlo, mhi) take theta from aux_f
    auto from_aux = [&](int pz) { return edge_plane_lo && (pz < mlo || pz >= mhi); };
    auto pull = [&](int pz, T (&raw)[L::Q]) {
        const int zz = wrapc(pz, nm);
        if (D3) pull_raw<L, ST>(p, fin, it.x, it.y, zz, raw);
        else pull_raw<L, ST>(p, fin, it.x, zz, 0, raw);
    };

    // prologue: frames of planes z0 - 4 .. z0 + 2, populations of plane z0 - 1
    {
        uint32_t w[FPT];
        for (int k = 0; k < 7; ++k) {
            fetch_frames(it.z0 - 4 + k, w);
            store_frames(it.z0 - 4 + k, w);
        }
    }
    T raw[L::Q];
#pragma unroll
    for (int i = 0; i < L::Q; ++i) raw[i] = T(0);
    if (PREFETCH && !from_aux(it.z0 - 1)) pull(it.z0 - 1, raw);
    lds_barrier();

    float A[L::Q], B[L::Q];
    Frame fa = {1.f, 0.f}, fb = {1.f, 0.f};
#pragma unroll
    for (int i = 0; i < L::Q; ++i) A[i] = B[i] = 0.f;

    for (int pz = it.z0 - 1; pz <= it.z1; ++pz) {
        // 1. decode plane pz into B (own frame and source frames from LDS), its theta
        float thv;
        if (from_aux(pz)) {
            const long long c = D3 ? ((long long)pz * p.ny + it.y) * p.nx + it.x : (long long)pz * p.nx + it.x;
            thv = aux_f[c];
        } else {
            constexpr int H = D3 ? 3 : 0;  // halo rows of the frame region (none in 2D)
            if (!PREFETCH) pull(pz, raw);
            fb = unpack_frame(frs[slot7(pz)][ty + H][tx + 3]);
            const FrameRef<L> ref = frame_ref<L>(fb);
            B[0] = Codec<ST>::dec(raw[0], p.dref[0]);
#pragma unroll
            for (int i = 1; i < L::Q; ++i) {
                const int cm = D3 ? L::cz[i] : L::cy[i];
                const int cl = D3 ? L::cy[i] : 0;
                const Frame fs = unpack_frame(frs[slot7(pz - cm)][ty + H - cl][tx + 3 - L::cx[i]]);
                B[i] = Codec<ST>::dec(raw[i], p.dref[i]) + frame_shift<L>(ref, L::shell[i], fs);
            }
            float dr, j[3], ed;
            moments<L>(B, dr, j, ed);
            const float z3[3] = {0.f, 0.f, 0.f};
            Macro mq;
            macro_from_moments<L, false>(p, fb, dr, j, ed, z3, mq);
            thv = theta_field(p, fb, mq);
        }
        th[pz & 3][ty][tx] = thv;
        uint32_t w[FPT];
        fetch_frames(pz + 4, w);
        lds_barrier();
        // 2. loads of plane pz + 1, in flight during the collision
        if (PREFETCH && pz + 1 <= it.z1 && !from_aux(pz + 1)) pull(pz + 1, raw);
        // 3. collide plane pz - 1
        const int q = pz - 1;
        if (q >= it.z0 && it.interior) march_collide<L, ST, TY, TX>(p, fout, th, tx, ty, it.x, it.y, q, nm, A, fa);
        // 4. frames of plane pz + 4 replace those of pz - 3; rotate the planes
        store_frames(pz + 4, w);
#pragma unroll
        for (int i = 0; i < L::Q; ++i) A[i] = B[i];
        fa = fb;
        lds_barrier();
    }
}

// Variant table.  3D: tiles of (TX-2) x (TY-2) interior cells; 2D: strips of
// TX-2 cells; chunks of 32 or 64 planes along the march axis.
template <class L>
struct MarchVariants;

template <>
struct MarchVariants<D3Q39> {
    static constexpr int N = 3;
};
template <>
struct MarchVariants<D2Q37> {
    static constexpr int N = 3;
};

// KIND: 3 = k_march3 with the loads of the next plane in flight during the
// collision (more registers), 4 = without
template <class L, int ST, class S, int KIND>
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
    hipLaunchKernelGGL((k_march3<L, ST, S, KIND == 3>), dim3(ntx * nty * nch), block, 0, c.stream, p,
                       (const T*)c.pop_in, (T*)c.pop_out, c.aux_f, ntx, nty, mlo, mhi, chunk);
    return hipGetLastError();
}

inline int march_num_variants(const LaunchCtx& c)
{
    if (c.family != FAM_THERMAL) return 0;
    return c.lattice == 1 ? MarchVariants<D3Q39>::N : MarchVariants<D2Q37>::N;
}

// Library variants 3.. are the marching kernels 1.. of the table below.
inline bool march_variant_supported(const LaunchCtx& c, int lib_variant)
{
    const int v = lib_variant - 2;
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
    // {TX, TY, kind, waves per SIMD} of each variant, as launched by march_step
    static const int s3[4][4] = {{0, 0, 0, 0}, {34, 14, 3, 2}, {34, 10, 3, 2}, {34, 10, 4, 3}};
    static const int s2[4][4] = {{0, 0, 0, 0}, {258, 1, 3, 2}, {130, 1, 3, 2}, {130, 1, 4, 3}};
    const int* e = L::D == 3 ? s3[v] : s2[v];
    snprintf(name, len, "k_march3<%s,%d,MarchShape<%d,%d,%d>,%s>", lat, st, e[0], e[1], e[3],
             e[2] == 3 ? "true" : "false");
}

// Collide planes [mlo, mhi) along the last axis with the marching kernel of
// the context's variant.
template <class L, int ST, int FAM>
hipError_t march_step(const LaunchCtx& c, int mlo, int mhi)
{
    if (FAM != FAM_THERMAL || !march_variant_supported(c, c.variant)) return hipErrorNotSupported;
    if constexpr (L::D == 3) {
        switch (c.variant - 2) {
        case 1: return launch_march_shape<L, ST, MarchShape<34, 14, 2>, 3>(c, 32, mlo, mhi);
        case 2: return launch_march_shape<L, ST, MarchShape<34, 10, 2>, 3>(c, 64, mlo, mhi);
        case 3: return launch_march_shape<L, ST, MarchShape<34, 10, 3>, 4>(c, 32, mlo, mhi);
        }
    } else {
        switch (c.variant - 2) {
        case 1: return launch_march_shape<L, ST, MarchShape<258, 1, 2>, 3>(c, 64, mlo, mhi);
        case 2: return launch_march_shape<L, ST, MarchShape<130, 1, 2>, 3>(c, 32, mlo, mhi);
        case 3: return launch_march_shape<L, ST, MarchShape<130, 1, 3>, 4>(c, 32, mlo, mhi);
        }
    }
    return hipErrorNotSupported;
}

}  // namespace holb
