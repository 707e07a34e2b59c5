// Per-cell device code shared by every kernel variant: pull streaming, wall
// closure, shifted moments, stencil sources and the fused collision.
#pragma once

#include <hip/hip_runtime.h>

#include "holb_device.h"
#include "holb_wall.h"

namespace holb {

// Order in which blocks take cells.  The eight XCDs receive blocks round-
// robin (block b runs on XCD b % 8), each with its own L2.
//   band = 0: cell order -- the chip sweeps the domain plane by plane;
//   band < 0: each XCD gets a contiguous eighth of the cells;
//   band = G > 0: the chip still sweeps plane by plane, but each XCD takes
//     runs of G consecutive blocks (a band of rows of the plane), so the
//     rows a pull reaches mostly sit in the same L2.
// Orders other than 0 need a block count that is a multiple of 8 (of 8 G for
// bands); otherwise cell order is used.
__device__ __forceinline__ int xcd_block(int band = -1)
{
    const int nb = gridDim.x, b = blockIdx.x;
    if (band == 0 || nb % 8) return b;
    if (band < 0) return (b % 8) * (nb / 8) + b / 8;
    if (nb % (8 * band)) return b;
    const int j = b / 8, x = b % 8;
    return ((j / band) * 8 + x) * band + j % band;
}

template <class L>
__device__ __forceinline__ void cell_coords(const KParams& p, int cell, int& x, int& y, int& z)
{
    const unsigned r = fastdiv((unsigned)cell, p.div_nx);
    x = cell - (int)r * p.nx;
    const unsigned q = fastdiv(r, p.div_ny);
    y = (int)r - (int)q * p.ny;
    z = (int)q;
}

// Pull the Q populations of node (x, y, z) into the node's own frame fo (read
// from the frame plane of fin at the node).  Along the wall-normal axis of a
// walled domain, sources outside [0, n) are not read; their bits are
// returned.  Nodes at least 3 cells from every edge take the source of
// population i at cell - shift_i with a wave-uniform shift, so that each load
// is a uniform base plus one shared per-lane offset; the others wrap per
// coordinate.  WALLS = false compiles the periodic pull only.
// Load at a 32-bit byte offset from a base pointer (a wave-uniform base
// lets the load take the scalar-base + lane-offset addressing form).
template <class T>
__device__ __forceinline__ T load_at(const T* __restrict__ base, unsigned byte_off)
{
    return *(const T*)((const char*)base + byte_off);
}

// The same with the base made opaque by an empty asm (which also pins it to
// scalar registers), for the population loads of the interior pull, whose
// bases differ per population: otherwise the compiler folds each base into
// a per-lane 64-bit address, one or two vector instructions per load
// (quarter-rate multiply-adds among them).  The base must be the same on all
// lanes of a wavefront.  Only for loads that are all issued before any is
// consumed: the asm also keeps the scheduler from moving a load across it.
template <class T>
__device__ __forceinline__ T load_uniform_at(const T* __restrict__ base, unsigned byte_off)
{
    using GT = const __attribute__((address_space(1))) T;
    using GC = const __attribute__((address_space(1))) char;
    GT* g = (GT*)base;
    asm("" : "+s"(g));
    return *(GT*)((GC*)g + byte_off);
}

// Non-temporal store at a 32-bit byte offset from a wave-uniform base, made
// opaque in the same way (the stores of a node go to Q different planes).
template <class T>
__device__ __forceinline__ void store_nt_at(T* __restrict__ base, unsigned byte_off, T v)
{
    using GT = __attribute__((address_space(1))) T;
    using GC = __attribute__((address_space(1))) char;
    GT* g = (GT*)base;
    asm("" : "+s"(g));
    __builtin_nontemporal_store(v, (GT*)((GC*)g + byte_off));
}

// Frame of the plane m along the last axis (FM_PLANE).
__device__ __forceinline__ Frame plane_frame_of(const KParams& p, int m)
{
    Frame F;
    F.rho = p.plane_frame[2 * m];
    F.thb = p.plane_frame[2 * m + 1];
    return F;
}

// A wavefront on a wall layer (walled domains) whose lanes all lie at least
// 3 cells from the edges along the wall and in one plane along the normal.
template <class L>
__device__ __forceinline__ bool wall_layer_wave(const KParams& p, int x, int y, int z)
{
    const bool lat = x >= 3 && x < p.nx - 3 && (L::D == 2 || (y >= 3 && y < p.ny - 3));
    const int m = L::D == 3 ? z : y;
    return __all(lat && m == __builtin_amdgcn_readfirstlane(m));
}

// MOM1 (FM_CELLU): load the momentum words with the first phase (for
// kernels with few registers of their own) instead of in a second phase.
template <class L, int ST, bool WALLS, int FM, bool MOM1 = false, bool ISO = false>
__device__ __forceinline__ uint64_t pull_cell(const KParams& p, const typename Codec<ST>::T* __restrict__ fin,
                                              int x, int y, int z, float (&f)[L::Q], Frame& fo)
{
    using T = typename Codec<ST>::T;
    constexpr bool CF = FM != FM_PLANE;
    constexpr bool CU = FM == FM_CELLU;
    using FW = uint32_t;
    const FW* __restrict__ fp = frame_plane<ST>(fin, p.pitch, L::Q);
    [[maybe_unused]] const uint32_t* __restrict__ mp = fp + mom_offset(p.N);
    [[maybe_unused]] uint32_t mw[L::Q];
    const int cell = (z * p.ny + y) * p.nx + x;
    const bool inner_yz = y >= 3 && y < p.ny - 3 && (L::D == 2 || (z >= 3 && z < p.nz - 3));
    const bool inner = inner_yz && x >= 3 && x < p.nx - 3;
    // All addresses first, then all loads, then the arithmetic, so that the
    // 2Q loads of a node are in flight together.  The three cases are taken
    // per wavefront: every lane away from the edges (a wave-uniform base per
    // population and one shared lane offset), only the x edge in reach on an
    // x axis of at least 3 cells (a periodic correction of x per population),
    // or the general wrap with the wall bookkeeping.
    T raw[L::Q];
    FW fw[L::Q];
    uint64_t unk = 0;
    if (__all(inner)) {
        const unsigned cb = (unsigned)cell * (unsigned)sizeof(T), cf = (unsigned)cell * (unsigned)sizeof(FW);
#pragma unroll
        for (int i = 0; i < L::Q; ++i) {
            const int shift = (L::cz[i] * p.ny + L::cy[i]) * p.nx + L::cx[i];
            raw[i] = load_uniform_at(fin + ((long long)i * p.pitch - shift), cb);
            if (CF) fw[i] = load_at(fp - shift, cf);
            if (CU && MOM1) mw[i] = load_at(mp - shift, cf);
        }
        __builtin_amdgcn_sched_barrier(0);
    } else if (p.nx >= 3 && __all(inner_yz)) {
        // one correction of x either way: exact for axes of 3 cells or more
        // (|c_x| <= 3); shorter x axes take the general wrap below
#pragma unroll
        for (int i = 0; i < L::Q; ++i) {
            int src = cell - ((L::cz[i] * p.ny + L::cy[i]) * p.nx + L::cx[i]);
            if (L::cx[i] > 0 && x < L::cx[i]) src += p.nx;
            if (L::cx[i] < 0 && x >= p.nx + L::cx[i]) src -= p.nx;
            raw[i] = load_at(fin + (long long)i * p.pitch, (unsigned)src * (unsigned)sizeof(T));
            if (CF) fw[i] = load_at(fp, (unsigned)src * (unsigned)sizeof(FW));
            if (CU && MOM1) mw[i] = load_at(mp, (unsigned)src * 4u);
        }
        __builtin_amdgcn_sched_barrier(0);
    } else if (WALLS && p.walls && wall_layer_wave<L>(p, x, y, z)) {
        // a wall layer, every lane away from the edges along the wall and in
        // one plane: a population whose source plane lies beyond the wall is
        // unknown for the whole wavefront and is not read; the others take
        // the interior addressing
        const int m = L::D == 3 ? z : y, nm = L::D == 3 ? p.nz : p.ny;
        const unsigned cb = (unsigned)cell * (unsigned)sizeof(T), cf = (unsigned)cell * (unsigned)sizeof(FW);
#pragma unroll
        for (int i = 0; i < L::Q; ++i) {
            const int ms = m - (L::D == 3 ? L::cz[i] : L::cy[i]);
            if (ms >= 0 && ms < nm) {
                const int shift = (L::cz[i] * p.ny + L::cy[i]) * p.nx + L::cx[i];
                raw[i] = load_uniform_at(fin + ((long long)i * p.pitch - shift), cb);
                if (CF) fw[i] = load_at(fp - shift, cf);
                if (CU && MOM1) mw[i] = load_at(mp - shift, cf);
            } else {
                unk |= 1ull << i;
                raw[i] = T(0);
                if (CF) fw[i] = 0u;
                if (CU && MOM1) mw[i] = 0u;
            }
        }
        __builtin_amdgcn_sched_barrier(0);
    } else {
        const bool walls = WALLS && p.walls;
        int xs[7], ys[7], zs[7];
#pragma unroll
        for (int k = 0; k < 7; ++k) {
            xs[k] = wrapc(x + k - 3, p.nx);
            ys[k] = (L::D == 2 && walls) ? y + k - 3 : wrapc(y + k - 3, p.ny);
            zs[k] = (L::D == 3) ? (walls ? z + k - 3 : wrapc(z + k - 3, p.nz)) : 0;
        }
#pragma unroll
        for (int i = 0; i < L::Q; ++i) {
            const int sx = xs[3 - L::cx[i]], sy = ys[3 - L::cy[i]], sz = zs[3 - L::cz[i]];
            bool known = true;
            if (walls) {
                const int kw = (L::D == 2) ? sy : sz;
                const int nw = (L::D == 2) ? p.ny : p.nz;
                known = (kw >= 0 && kw < nw);
            }
            // an unknown population reads the node's own slot; the value is discarded
            const int src = known ? (sz * p.ny + sy) * p.nx + sx : cell;
            if (!known) unk |= 1ull << i;
            raw[i] = load_at(fin + (long long)i * p.pitch, (unsigned)src * (unsigned)sizeof(T));
            if (CF) fw[i] = load_at(fp, (unsigned)src * (unsigned)sizeof(FW));
            if (CU && MOM1) mw[i] = load_at(mp, (unsigned)src * 4u);
        }
    }
    // keep the scheduler from sinking loads into the arithmetic below
    __builtin_amdgcn_sched_barrier(0);
    f[0] = Codec<ST>::dec(raw[0], p.dref[0]);
    if constexpr (CF) {
        fo = unpack_frame(fw[0]);
        if constexpr (ISO) {
            // isothermal: every frame has theta_F = 1, where R_s(S) - R_s(O)
            // is rho_S - rho_O exactly (the general form below gives the same
            // bits there)
#pragma unroll
            for (int i = 1; i < L::Q; ++i) {
                const float v = Codec<ST>::dec(raw[i], p.dref[i]) + (unpack_frame(fw[i]).rho - fo.rho);
                f[i] = (WALLS && ((unk >> i) & 1ull)) ? 0.0f : v;
            }
        } else {
            const FrameRef<L> ref = frame_ref<L>(fo);
#pragma unroll
            for (int i = 1; i < L::Q; ++i) {
                const float v = Codec<ST>::dec(raw[i], p.dref[i]) +
                                frame_shift<L>(ref, L::shell[i], unpack_frame(fw[i]));
                f[i] = (WALLS && ((unk >> i) & 1ull)) ? 0.0f : v;
            }
        }
    } else {
        // plane frames: the shift depends only on the plane, the last-axis
        // velocity and the shell (zero within the plane)
        const int m = L::D == 3 ? z : y;
        fo = plane_frame_of(p, m);
        const float* __restrict__ sh = p.plane_shift + (long long)m * 7 * L::NS;
#pragma unroll
        for (int i = 1; i < L::Q; ++i) {
            const int cm = L::D == 3 ? L::cz[i] : L::cy[i];
            float v = Codec<ST>::dec(raw[i], p.dref[i]);
            if (cm != 0) v += sh[(cm + 3) * L::NS + L::shell[i]];
            f[i] = (WALLS && ((unk >> i) & 1ull)) ? 0.0f : v;
        }
    }
    if constexpr (CU) {
        // Second load phase: the momentum words of the same sources, whose
        // part c_i . P_S of the source's frame is added back.  Loading them
        // with the first phase would hold 3Q words in flight and cost a wave
        // of occupancy.
        if (MOM1) {
        } else if (__all(inner)) {
            const unsigned cf = (unsigned)cell * 4u;
#pragma unroll
            for (int i = 1; i < L::Q; ++i) {
                const int shift = (L::cz[i] * p.ny + L::cy[i]) * p.nx + L::cx[i];
                mw[i] = load_at(mp - shift, cf);
            }
        } else {
#pragma unroll
            for (int i = 1; i < L::Q; ++i) {
                const int sx = wrap_seq(x - L::cx[i], p.nx);
                int sy = y - L::cy[i], sz = z - L::cz[i];
                if (L::D == 2) {
                    sz = 0;
                    sy = (WALLS && p.walls) ? min(max(sy, 0), p.ny - 1) : wrap_seq(sy, p.ny);
                } else {
                    sy = wrap_seq(sy, p.ny);
                    sz = (WALLS && p.walls) ? min(max(sz, 0), p.nz - 1) : wrap_seq(sz, p.nz);
                }
                // an unknown population reads a clamped slot; its value is discarded
                mw[i] = load_at(mp, (unsigned)((sz * p.ny + sy) * p.nx + sx) * 4u);
            }
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int i = 1; i < L::Q; ++i)
            if (!(WALLS && ((unk >> i) & 1ull))) f[i] += cdot_mom<L>(i, mw[i]);
    }
    return unk;
}

// Store the post-collision populations of a node; they are read once, by
// the next step's pulls, so they are written non-temporally (without
// allocating in the caches); the frame words, which every puller of a cell
// reads, are written normally.  FM_CELL: in a new frame
// fn (written to the frame plane of fout), h_i(fn) = h_i(fo) + R_i(fo) -
// R_i(fn), one shift per shell.  FM_CELLU: the same, minus c_i . P of the
// node's new momentum word.  FM_PLANE: the frame of the plane is fixed, the
// values are stored as they are.
template <class L, int ST, int FM>
__device__ __forceinline__ void store_cell(const KParams& p, typename Codec<ST>::T* __restrict__ fout, long long cell,
                                           float (&f)[L::Q], const Frame& fo, float rho, float thb,
                                           const float (&u)[3])
{
    // wave-uniform plane bases and one shared lane offset: the address of
    // each store costs no vector instructions
    const unsigned cb = (unsigned)cell * (unsigned)sizeof(typename Codec<ST>::T);
    if constexpr (FM == FM_CELLU) {
        const uint32_t packed = pack_frame(rho, thb);
        float P[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) P[a] = a < L::D ? rho * fmaf(u[a], Lat<L>::ic0sq, -p.u0s[a]) : 0.0f;
        const uint32_t mom = pack_mom(P);
        uint32_t* fpo = frame_plane<ST>(fout, p.pitch, L::Q);
        fpo[cell] = packed;
        fpo[mom_offset(p.N) + cell] = mom;
        const Frame fn = unpack_frame(packed);
        const FrameRef<L> ref = frame_ref<L>(fo);
        float sh[L::NS];  // R(fo) - R(fn)
#pragma unroll
        for (int s = 0; s < L::NS; ++s) sh[s] = -frame_shift<L>(ref, s, fn);
        store_nt_at(fout, cb, Codec<ST>::enc(f[0] + sh[0], p.dref[0]));
        // +/-c pairs share c . P with opposite signs
#pragma unroll
        for (int i = 1; i < L::Q; i += 2) {
            const float cp = cdot_mom<L>(i, mom);
            const float s = sh[L::shell[i]];
            store_nt_at(fout + (long long)i * p.pitch, cb, Codec<ST>::enc(f[i] + s - cp, p.dref[i]));
            store_nt_at(fout + (long long)(i + 1) * p.pitch, cb, Codec<ST>::enc(f[i + 1] + s + cp, p.dref[i + 1]));
        }
    } else if constexpr (FM == FM_CELL) {
        const uint32_t packed = pack_frame(rho, thb);
        frame_plane<ST>(fout, p.pitch, L::Q)[cell] = packed;
        const Frame fn = unpack_frame(packed);
        const FrameRef<L> ref = frame_ref<L>(fo);
        float sh[L::NS];  // R(fo) - R(fn)
#pragma unroll
        for (int s = 0; s < L::NS; ++s) sh[s] = -frame_shift<L>(ref, s, fn);
#pragma unroll
        for (int i = 0; i < L::Q; ++i)
            store_nt_at(fout + (long long)i * p.pitch, cb, Codec<ST>::enc(f[i] + sh[L::shell[i]], p.dref[i]));
    } else {
#pragma unroll
        for (int i = 0; i < L::Q; ++i) store_nt_at(fout + (long long)i * p.pitch, cb, Codec<ST>::enc(f[i], p.dref[i]));
    }
}

template <class L>
__device__ __forceinline__ void wall_coord(const KParams& p, int x, int y, int z, int& kw, int& nw, int& cil)
{
    if (L::D == 2) { kw = y; nw = p.ny; cil = x; }
    else { kw = z; nw = p.nz; cil = x + p.nx * y; }
}

// Pull + wall closure + deviation moments in the node's frame fo (dr = rho -
// rho_F, j, ed = e - rho_F D c0^2 theta_F; no stencil force yet).  Shared by
// every pass over the state so that they agree bitwise.  f holds the
// deviations h_i.  WALLS = false compiles out the wall closure (periodic
// domains and interior planes).
template <class L, int ST, bool WALLS, int FM, bool MOM1 = false, bool ISO = false>
__device__ __forceinline__ void load_state(const KParams& p, const typename Codec<ST>::T* __restrict__ fin,
                                           const double* __restrict__ tgt_in, int x, int y, int z,
                                           float (&f)[L::Q], Frame& fo, float& dr, float (&j)[3], float& ed)
{
    uint64_t unk = pull_cell<L, ST, WALLS, FM, MOM1, ISO>(p, fin, x, y, z, f, fo);
    if (WALLS && p.walls && unk) {
        // the closure of this state, solved before any pass (k_wall_fluid,
        // k_wall_solve): read its populations
        int kw, nw, cil;
        wall_coord<L>(p, x, y, z, kw, nw, cil);
        if (kw < 3) load_closed<L, 0>(p, kw, cil, f);
        else load_closed<L, 1>(p, nw - 1 - kw, cil, f);
    }
    moments<L>(f, dr, j, ed);
}

// Eq. (3.8): F^SC(x) = -G psi(x) sum_i w_i psi(x + c_i) c_i, FP64, periodic.
template <class L>
__device__ __forceinline__ void sc_force(const KParams& p, const double* __restrict__ psi, int x, int y, int z,
                                         double& psi_x, double (&F)[3])
{
    double acc[3] = {0.0, 0.0, 0.0};
    const int cell = (z * p.ny + y) * p.nx + x;
    // Sums in velocity order.  A wavefront whose lanes all lie at least 3
    // cells from every edge reads neighbour i at a wave-uniform base
    // psi + shift_i and one shared lane offset; the others wrap per coordinate.
    auto add = [&](int i, double v) {
        const double ps = v * L::shell_w[L::shell[i]];
        if (L::cx[i]) acc[0] = fma((double)L::cx[i], ps, acc[0]);
        if (L::cy[i]) acc[1] = fma((double)L::cy[i], ps, acc[1]);
        if (L::cz[i]) acc[2] = fma((double)L::cz[i], ps, acc[2]);
    };
    const bool inner = x >= 3 && x < p.nx - 3 && y >= 3 && y < p.ny - 3 && (L::D == 2 || (z >= 3 && z < p.nz - 3));
    if (__all(inner)) {
        const unsigned cb = (unsigned)cell * (unsigned)sizeof(double);
#pragma unroll
        for (int i = 1; i < L::Q; ++i) add(i, load_at(psi + (L::cz[i] * p.ny + L::cy[i]) * p.nx + L::cx[i], cb));
    } else {
#pragma unroll
        for (int i = 1; i < L::Q; ++i) {
            const int sx = wrapc(x + L::cx[i], p.nx), sy = wrapc(y + L::cy[i], p.ny);
            const int sz = L::D == 3 ? wrapc(z + L::cz[i], p.nz) : 0;
            add(i, psi[(sz * p.ny + sy) * p.nx + sx]);
        }
    }
    psi_x = psi[cell];
#pragma unroll
    for (int a = 0; a < 3; ++a) F[a] = -p.G * psi_x * acc[a];
}

// Pressure-tensor coefficient of Eq. (3.12) from F^SC and psi (FP64).
__device__ __forceinline__ float ptensor_coef(const KParams& p, double psi_x, const double (&F)[3])
{
    const double F2 = F[0] * F[0] + F[1] * F[1] + F[2] * F[2];
    return (float)(p.pfac * F2 / (psi_x * psi_x));
}

// Section 3.2: grad theta by central differences; one-sided first differences
// on the wall layers of a walled domain.
template <class L>
__device__ __forceinline__ void grad_theta(const KParams& p, const float* __restrict__ th, int x, int y, int z,
                                           float (&g)[3])
{
    g[2] = 0.0f;
    // A wavefront with every lane off the edges of the other axes takes their
    // central differences at wave-uniform bases and one shared lane offset;
    // x wraps by a select.
    const bool inner_yz = y >= 1 && y < p.ny - 1 && (L::D == 2 || (z >= 1 && z < p.nz - 1));
    if (__all(inner_yz)) {
        const int cell = (z * p.ny + y) * p.nx + x;
        const unsigned cb = (unsigned)cell * 4u;
        const int row = cell - x;
        const int xp = x + 1 < p.nx ? x + 1 : 0, xm = x > 0 ? x - 1 : p.nx - 1;
        g[0] = 0.5f * (th[row + xp] - th[row + xm]);
        g[1] = 0.5f * (load_at(th + p.nx, cb) - load_at(th - p.nx, cb));
        if (L::D == 3) g[2] = 0.5f * (load_at(th + p.nx * p.ny, cb) - load_at(th - p.nx * p.ny, cb));
        return;
    }
    auto at = [&](int xx, int yy, int zz) { return th[(zz * p.ny + yy) * p.nx + xx]; };
    g[0] = 0.5f * (at(wrapc(x + 1, p.nx), y, z) - at(wrapc(x - 1, p.nx), y, z));
    if (L::D == 2) {
        if (p.walls) {
            if (y == 0) g[1] = at(x, 1, z) - at(x, 0, z);
            else if (y == p.ny - 1) g[1] = at(x, y, z) - at(x, y - 1, z);
            else g[1] = 0.5f * (at(x, y + 1, z) - at(x, y - 1, z));
        } else {
            g[1] = 0.5f * (at(x, wrapc(y + 1, p.ny), z) - at(x, wrapc(y - 1, p.ny), z));
        }
    } else {
        g[1] = 0.5f * (at(x, wrapc(y + 1, p.ny), z) - at(x, wrapc(y - 1, p.ny), z));
        if (p.walls) {
            if (z == 0) g[2] = at(x, y, 1) - at(x, y, 0);
            else if (z == p.nz - 1) g[2] = at(x, y, z) - at(x, y, z - 1);
            else g[2] = 0.5f * (at(x, y, z + 1) - at(x, y, z - 1));
        } else {
            g[2] = 0.5f * (at(x, y, wrapc(z + 1, p.nz)) - at(x, y, wrapc(z - 1, p.nz)));
        }
    }
}

// The state of a node on the wall layers, kept for the next step's closure
// (targets of Eq. 4.7).  Density and temperature are stored in FP64 as
// frame + deviation, without the FP32 rounding of the sum: the closure
// reflects them about the wall values and is sensitive to their last bits.
template <class L>
__device__ __forceinline__ void write_targets(const KParams& p, double* __restrict__ tgt_out, int x, int y, int z,
                                              const Frame& fo, const Macro& m)
{
    int kw, nw, cil;
    wall_coord<L>(p, x, y, z, kw, nw, cil);
    const int slot = wall_slot(kw, nw);
    if (slot < 0) return;
    double* t = tgt_out + (long long)slot * (L::D + 2) * p.nlayer + cil;
    t[0] = (double)fo.rho + (double)m.dr;
#pragma unroll
    for (int a = 0; a < L::D; ++a) t[(long long)(1 + a) * p.nlayer] = m.u[a];
    t[(long long)(1 + L::D) * p.nlayer] = (p.flags & KF_ISO) ? 1.0 : (1.0 + (double)fo.thb) + (double)m.dth;
}

// A wall node keeps the target it was closed at as the starting point of the
// next step's solve (warm slot of the targets).
template <class L>
__device__ __forceinline__ void write_warm_start(const KParams& p, double* __restrict__ tgt_out, int x, int y, int z)
{
    int kw, nw, cil;
    wall_coord<L>(p, x, y, z, kw, nw, cil);
    if (kw != 0 && kw != nw - 1) return;
    const int side = kw == 0 ? 0 : 1;
    const double* ws = p.wsol + (long long)side * WSOL_COMPS * p.nlayer + cil;
    double* t = tgt_out + (long long)warm_slot(side) * (L::D + 2) * p.nlayer + cil;
    t[0] = ws[0];
#pragma unroll
    for (int a = 0; a < L::D; ++a) t[(long long)(1 + a) * p.nlayer] = ws[(long long)(1 + a) * p.nlayer];
    t[(long long)(1 + L::D) * p.nlayer] = ws[4 * (long long)p.nlayer];
    double* lu = tgt_out + tgt_lu_offset(L::D, side, p.nlayer) + cil;
#pragma unroll
    for (int k = 0; k < 16; ++k) lu[(long long)k * p.nlayer] = ws[(long long)(5 + k) * p.nlayer];
}

// Stencil force of the pressure-tensor family (F^SC in FP32 and the
// coefficient of Eq. 3.12); zero for the other families.
template <class L, int FAM>
__device__ __forceinline__ void stencil_force(const KParams& p, const double* __restrict__ aux_d, int x, int y,
                                              int z, float (&Fext)[3], float& pc)
{
#pragma unroll
    for (int a = 0; a < 3; ++a) Fext[a] = 0.0f;
    pc = 0.0f;
    if (FAM == FAM_PTENSOR) {
        double psi_x, Fsc[3];
        sc_force<L>(p, aux_d, x, y, z, psi_x, Fsc);
#pragma unroll
        for (int a = 0; a < 3; ++a) Fext[a] = (float)Fsc[a];
        pc = ptensor_coef(p, psi_x, Fsc);
    }
}

template <class L, int ST, int FAM>
__device__ __forceinline__ void full_macro(const KParams& p, const Frame& fo, const float* __restrict__ aux_f,
                                           const double* __restrict__ aux_d, int x, int y, int z, float dr,
                                           const float (&j)[3], float ed, Macro& m, float& pc)
{
    float Fext[3];
    stencil_force<L, FAM>(p, aux_d, x, y, z, Fext, pc);
    macro_from_moments<L>(p, fo, dr, j, ed, Fext, m);
}


// Temperature field value of a node for the gradient stencil: theta minus
// the global reference theta0, from the frame offset and the deviation.
__device__ __forceinline__ float theta_field(const KParams& p, const Frame& fo, const Macro& m)
{
    return (fo.thb - p.thb_ref) + m.dth;
}

// One full step of one cell: pull, closure, moments, sources, collision and
// store of the post-collision populations at `cell` of fout.
template <class L, int ST, int FAM, bool WALLS, int FM, bool ISO = false>
__device__ __forceinline__ void step_cell(const KParams& p, const typename Codec<ST>::T* __restrict__ fin,
                                          typename Codec<ST>::T* __restrict__ fout, const float* __restrict__ aux_f,
                                          const double* __restrict__ aux_d, const double* __restrict__ tgt_in,
                                          double* __restrict__ tgt_out, int cell,
                                          float* __restrict__ theta_out = nullptr)
{
    using LL = Lat<L>;
    int x, y, z;
    cell_coords<L>(p, cell, x, y, z);
    // the psi stencil before the pull: its loads and sums are done before
    // the populations occupy the register file
    float Fext[3], pc;
    stencil_force<L, FAM>(p, aux_d, x, y, z, Fext, pc);
    float f[L::Q], dr, j[3], ed;
    Frame fo;
    load_state<L, ST, WALLS, FM, false, ISO>(p, fin, tgt_in, x, y, z, f, fo, dr, j, ed);
    Macro m;
    macro_from_moments<L>(p, fo, dr, j, ed, Fext, m);
    if (WALLS && p.walls) {
        write_targets<L>(p, tgt_out, x, y, z, fo, m);
        write_warm_start<L>(p, tgt_out, x, y, z);
    }
    float gT[3] = {0.f, 0.f, 0.f};
    float hc = 0.0f;
    if (FAM == FAM_THERMAL) {
        grad_theta<L>(p, aux_f, x, y, z, gT);
        hc = p.hfac * m.rho * m.theta;
        // with the previous step's gradient: this step's theta field, for the
        // next step (the value the field pass would compute)
        if (theta_out) theta_out[cell] = theta_field(p, fo, m);
    }
    collide<L, ST == ST_F32>(p, fo, f, m, hc, gT, pc);
    store_cell<L, ST, FM>(p, fout, cell, f, fo, m.rho, m.thb, m.u);
}

// Field pass of one cell: theta (thermal family) or psi (pressure-tensor
// family) of the current state, read by the stencil of the following pass.
template <class L, int ST, int FAM, bool WALLS, int FM, bool ISO = false>
__device__ __forceinline__ void aux_cell(const KParams& p, const typename Codec<ST>::T* __restrict__ fin,
                                         const double* __restrict__ tgt_in, float* __restrict__ aux_f,
                                         double* __restrict__ aux_d, int cell)
{
    int x, y, z;
    cell_coords<L>(p, cell, x, y, z);
    float f[L::Q], dr, j[3], ed;
    Frame fo;
    load_state<L, ST, WALLS, FM, true, ISO>(p, fin, tgt_in, x, y, z, f, fo, dr, j, ed);
    if (FAM == FAM_PTENSOR) {
        bool bad = false;
        aux_d[cell] = psi_eos(p, (double)fo.rho + (double)dr, L::c0sq, bad);
        if (bad) raise_err(p, HOLB_ERR_EOS_BIT);
    } else {
        const float z3[3] = {0.f, 0.f, 0.f};
        Macro m;
        macro_from_moments<L>(p, fo, dr, j, ed, z3, m);
        aux_f[cell] = theta_field(p, fo, m);
    }
}

// Initial frame of one cell (written before the populations, which are
// stored in the frames of the cells they are pulled from).
template <class L, int ST, int FM>
__device__ __forceinline__ void init_frame_cell(const KParams& p, const float* __restrict__ rho,
                                                const float* __restrict__ u, const float* __restrict__ theta,
                                                typename Codec<ST>::T* __restrict__ fout, int cell)
{
    const float thb = (p.flags & KF_ISO) ? 0.0f : theta[cell] - 1.0f;
    const uint32_t packed = pack_frame(rho[cell], thb);
    if constexpr (FM == FM_CELLU) {
        float P[3];
#pragma unroll
        for (int a = 0; a < 3; ++a)
            P[a] = a < L::D ? rho[cell] * fmaf(u[(long long)a * p.N + cell], Lat<L>::ic0sq, -p.u0s[a]) : 0.0f;
        uint32_t* fpo = frame_plane<ST>(fout, p.pitch, L::Q);
        fpo[cell] = packed;
        fpo[mom_offset(p.N) + cell] = pack_mom(P);
    } else {
        frame_plane<ST>(fout, p.pitch, L::Q)[cell] = packed;
    }
}

// Initial state of one cell: f^0_i(x) = f^eq_i(rho, u, theta)(x), written to
// the slot x - c_i that the first pull of node x reads, in the frame of that
// slot's cell.
template <class L, int ST, int FM>
__device__ __forceinline__ void init_cell(const KParams& p, const float* __restrict__ rho,
                                          const float* __restrict__ u, const float* __restrict__ theta,
                                          typename Codec<ST>::T* __restrict__ fout, double* __restrict__ tgt, int cell)
{
    using LL = Lat<L>;
    int x, y, z;
    cell_coords<L>(p, cell, x, y, z);
    Macro m;
    m.rho = rho[cell];
    m.u[0] = m.u[1] = m.u[2] = 0.f;
#pragma unroll
    for (int a = 0; a < L::D; ++a) m.u[a] = u[(long long)a * p.N + cell];
    m.theta = (p.flags & KF_ISO) ? 1.0f : theta[cell];
    m.thb = m.theta - 1.0f;
    if (!(m.rho > 0.0f) || !(m.rho < 3.0e38f)) raise_err(p, HOLB_ERR_DENSITY_BIT);
    if (!(m.theta > 0.0f) || !(m.theta < 3.0e38f)) raise_err(p, HOLB_ERR_THETA_BIT);
    if (p.walls) {
        const Frame exact{m.rho, m.thb};  // the initial fields as they are: deviation 0
        Macro m0 = m;
        m0.dr = 0.0f;
        m0.dth = 0.0f;
        write_targets<L>(p, tgt, x, y, z, exact, m0);
        int kw, nw, cil;
        wall_coord<L>(p, x, y, z, kw, nw, cil);
        if (kw == 0 || kw == nw - 1) {
            double* t = tgt + (long long)warm_slot(kw == 0 ? 0 : 1) * (L::D + 2) * p.nlayer + cil;
            t[0] = m.rho;
#pragma unroll
            for (int a = 0; a < L::D; ++a) t[(long long)(1 + a) * p.nlayer] = m.u[a];
            t[(long long)(1 + L::D) * p.nlayer] = m.theta;
            double* lu = tgt + tgt_lu_offset(L::D, kw == 0 ? 0 : 1, p.nlayer) + cil;
#pragma unroll
            for (int k = 0; k < 16; ++k) lu[(long long)k * p.nlayer] = 0.0;  // no Jacobian yet
        }
    }
    const uint32_t* fp = frame_plane<ST>(fout, p.pitch, L::Q);
    const int mz = L::D == 3 ? z : y;
    const Frame fo = FM != FM_PLANE ? unpack_frame(fp[cell]) : plane_frame_of(p, mz);
    [[maybe_unused]] const FrameRef<L> ref = frame_ref<L>(fo);
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        int dx = wrapc(x - L::cx[i], p.nx);
        int dy, dz;
        bool inside = true;
        if (L::D == 2) {
            dz = 0;
            dy = y - L::cy[i];
            if (p.walls) inside = dy >= 0 && dy < p.ny;
            else dy = wrapc(dy, p.ny);
        } else {
            dy = wrapc(y - L::cy[i], p.ny);
            dz = z - L::cz[i];
            if (p.walls) inside = dz >= 0 && dz < p.nz;
            else dz = wrapc(dz, p.nz);
        }
        if (!inside) continue;
        const int slot = (dz * p.ny + dy) * p.nx + dx;
        if (p.walls) {
            // A population of this node that would leave through a wall has
            // a slot no node pulls; it holds the equilibrium the node would
            // send out, in the node's own frame (before the first step, the
            // closure balances the mass of these slots).
            const int mo = (L::D == 2 ? y : z) + cnorm<L>(i), nmo = L::D == 2 ? p.ny : p.nz;
            if (mo < 0 || mo >= nmo) {
                float ho = feq_dev<L>(fo, i, m.rho, m.u, m.thb);
                if constexpr (FM == FM_CELLU) ho -= cdot_mom<L>(i, fp[mom_offset(p.N) + cell]);
                fout[(long long)i * p.pitch + cell] = Codec<ST>::enc(ho, p.dref[i]);
            }
        }
        // in the node's own frame, then moved into the slot cell's frame
        const float fe = feq_dev<L>(fo, i, m.rho, m.u, m.thb);
        float h;
        if constexpr (FM == FM_CELL) {
            h = fe - frame_shift<L>(ref, L::shell[i], unpack_frame(fp[slot]));
        } else if constexpr (FM == FM_CELLU) {
            h = fe - frame_shift<L>(ref, L::shell[i], unpack_frame(fp[slot])) -
                cdot_mom<L>(i, fp[mom_offset(p.N) + slot]);
        } else {
            const int cm = L::D == 3 ? L::cz[i] : L::cy[i];
            h = cm == 0 ? fe : fe - p.plane_shift[((long long)mz * 7 + cm + 3) * L::NS + L::shell[i]];
        }
        fout[(long long)i * p.pitch + slot] = Codec<ST>::enc(h, p.dref[i]);
    }
}

}  // namespace holb
