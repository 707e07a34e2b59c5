// gfx950 kernels of the high-order lattice Boltzmann step and their launchers
// (templates; instantiated per lattice and storage set by holb_inst_*.hip).
//
// Data layout: populations are structure-of-arrays, Q planes of `pitch`
// elements (256-byte aligned), cell = x + nx * (y + ny * z).  The stored
// values are deviations from a frame (FrameMode in holb_params.h): per cell
// (binary16 pair rho, theta - 1 in a plane after the populations, with the
// momentum in a second plane for FM_CELLU) or fixed per plane along the last
// axis (a small table); the frame mode is chosen per configuration, for any
// storage width (holb_host.h).  The state buffer
// holds the post-collision populations of the last step; a step pulls
// f^_i(x) = buf[i][x - c_i] (streaming, left side of Eq. 4.4), applies the wall
// closure, forms the shifted moments (Eq. 4.5), the sources and the collision,
// and writes the post-collision populations of x into the other buffer.
//
// Generic variant: one cell per thread, 256-thread blocks along x.  Stencil
// sources (temperature gradient, pseudopotential force) read a field written
// by a preceding pass over the same state (launch_aux), or, for the
// temperature gradient with grad_lag, by the previous step's collision.
#pragma once

#include <hip/hip_runtime.h>
#include <stdio.h>

#include "holb_cell.h"
#include "holb_device.h"
#include "holb_internal.h"

namespace holb {

constexpr int GEN_BLOCK = 256;


// --------------------------------------------------------------- kernels

template <class L, int ST, int FM>
__global__ void __launch_bounds__(GEN_BLOCK)
k_init_frame(const KParams p, const float* __restrict__ rho, const float* __restrict__ u,
             const float* __restrict__ theta, typename Codec<ST>::T* __restrict__ fout)
{
    const int cell = xcd_block() * GEN_BLOCK + threadIdx.x;
    if (cell < p.N) init_frame_cell<L, ST, FM>(p, rho, u, theta, fout, cell);
}

template <class L, int ST, int FM>
__global__ void __launch_bounds__(GEN_BLOCK)
k_init(const KParams p, const float* __restrict__ rho, const float* __restrict__ u,
       const float* __restrict__ theta, typename Codec<ST>::T* __restrict__ fout, double* __restrict__ tgt)
{
    const int cell = xcd_block() * GEN_BLOCK + threadIdx.x;
    if (cell < p.N) init_cell<L, ST, FM>(p, rho, u, theta, fout, tgt, cell);
}

// Per-plane frames (FM_PLANE): the mean density and temperature of each plane
// along the last axis of the initial fields, FP64 sums; one block per plane.
template <int UNUSED = 0>
__global__ void __launch_bounds__(256)
k_plane_frames(const KParams p, const float* __restrict__ rho, const float* __restrict__ theta,
               float* __restrict__ frames)
{
    __shared__ double red[4][2];
    const long long c0 = (long long)blockIdx.x * p.nlayer;
    double sr = 0.0, st = 0.0;
    for (int k = threadIdx.x; k < p.nlayer; k += 256) {
        sr += (double)rho[c0 + k];
        st += (double)theta[c0 + k];
    }
    for (int off = 32; off > 0; off >>= 1) {
        sr += __shfl_xor(sr, off, 64);
        st += __shfl_xor(st, off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        red[threadIdx.x >> 6][0] = sr;
        red[threadIdx.x >> 6][1] = st;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const double r = ((red[0][0] + red[1][0]) + red[2][0]) + red[3][0];
        const double t = ((red[0][1] + red[1][1]) + red[2][1]) + red[3][1];
        frames[2 * blockIdx.x] = (float)(r / p.nlayer);
        frames[2 * blockIdx.x + 1] = (p.flags & KF_ISO) ? 0.0f : (float)(t / p.nlayer - 1.0);
    }
}

// Shift table of the per-plane frames: R_s(frame(m - c_m)) - R_s(frame(m)) for
// every plane m, last-axis velocity component c_m in [-3, 3] and shell s (zero where
// plane m - c_m lies beyond a wall: those populations are rebuilt, not read).
template <class L>
__global__ void k_plane_shift(const KParams p, const float* __restrict__ frames, float* __restrict__ shifts)
{
    const int m = blockIdx.x, t = threadIdx.x;
    if (t >= 7 * L::NS) return;
    const int cm = t / L::NS - 3, s = t % L::NS;
    const int nm = L::D == 3 ? p.nz : p.ny;
    int src = m - cm;
    float v = 0.0f;
    const bool inside = src >= 0 && src < nm;
    if (inside || !p.walls) {
        src = wrapc(src, nm);
        Frame O, S;
        O.rho = frames[2 * m]; O.thb = frames[2 * m + 1];
        S.rho = frames[2 * src]; S.thb = frames[2 * src + 1];
        const FrameRef<L> ref = frame_ref<L>(O);
        v = cm == 0 ? 0.0f : frame_shift<L>(ref, s, S);
    }
    shifts[((long long)m * 7 + (cm + 3)) * L::NS + s] = v;
}

// A set of planes along the last axis, [lo0, lo0 + n0) and [lo1, lo1 + n1):
// the whole domain, or the layers next to the walls.
struct PlaneSet {
    int lo0, n0, lo1, n1;
};

__device__ __forceinline__ int plane_cell(const KParams& p, const PlaneSet& ps, int c)
{
    const int k = (int)fastdiv((unsigned)c, p.div_layer), r = c - k * p.nlayer;
    const int plane = k < ps.n0 ? ps.lo0 + k : ps.lo1 + (k - ps.n0);
    return plane * p.nlayer + r;
}

// Wall closure, first half: the mass that the closure of the two fluid
// boundary layers next to each wall rebuilds (FP64), per column.
template <class L, int ST, int FM>
__global__ void __launch_bounds__(GEN_BLOCK)
k_wall_fluid(const KParams p, const typename Codec<ST>::T* __restrict__ fin, const double* __restrict__ tgt_in,
             float* __restrict__ theta_out)
{
    const int c = blockIdx.x * GEN_BLOCK + threadIdx.x;
    if (c >= 4 * p.nlayer) return;
    const int q = (int)fastdiv((unsigned)c, p.div_layer), cil = c - q * p.nlayer;
    const int side = q >> 1, d = 1 + (q & 1);
    const int nm = L::D == 3 ? p.nz : p.ny;
    const int k = side == 0 ? d : nm - 1 - d;
    int x, y, z;
    cell_coords<L>(p, k * p.nlayer + cil, x, y, z);
    float f[L::Q];
    Frame fo;
    pull_cell<L, ST, true, FM, true>(p, fin, x, y, z, f, fo);
    double t[5];
#pragma unroll
    for (int cc = 0; cc < L::D + 2; ++cc) t[cc] = tgt_in[((long long)wall_slot(k, nm) * (L::D + 2) + cc) * p.nlayer + cil];
    WallState after;
    p.mflu[(long long)q * p.nlayer + cil] = fluid_close<L>(p, fo, f, t, k, nm, after);
    if (side == 0) store_closed<L, 0>(p, d, cil, f);
    else store_closed<L, 1>(p, d, cil, f);
    // the temperature field of the gradient stencil on the wall layers
    if (theta_out) theta_out[k * p.nlayer + cil] = theta_field64(p, after);
}

// Absolute value (FP64) of the stored population j at cell, in the frame it
// was stored in.
template <class L, int ST, int FM>
__device__ __forceinline__ double stored_population(const KParams& p, const typename Codec<ST>::T* __restrict__ fin,
                                                    int j, int cell, int plane)
{
    double v = (double)Codec<ST>::dec(fin[(long long)j * p.pitch + cell], p.dref[j]);
    Frame F;
    if constexpr (FM == FM_PLANE) {
        F = plane_frame_of(p, plane);
    } else {
        const uint32_t* fp = frame_plane<ST>(fin, p.pitch, L::Q);
        F = unpack_frame(fp[cell]);
        if constexpr (FM == FM_CELLU) v += (double)cdot_mom<L>(j, fp[mom_offset(p.N) + cell]);
    }
    return L::shell_w[L::shell[j]] * (v + (double)F.rho * rest_bracket64<L>(L::shell[j], (double)F.thb));
}

// Wall closure, second half: the target of each wall node (see holb_wall.h).
template <class L, int ST, int FM, int SIDE>
__device__ __forceinline__ void wall_solve_cell(const KParams& p, const typename Codec<ST>::T* __restrict__ fin,
                                                const double* __restrict__ tgt_in, float* __restrict__ theta_out,
                                                int cil)
{
    constexpr int D = L::D;
    const int nm = D == 3 ? p.nz : p.ny;
    const int k0 = SIDE == 0 ? 0 : nm - 1;
    int x, y, z;
    cell_coords<L>(p, k0 * p.nlayer + cil, x, y, z);
    float f[L::Q];
    Frame fo;
    pull_cell<L, ST, true, FM, true>(p, fin, x, y, z, f, fo);
    const WallKnown K = wall_known<L, SIDE>(fo, f);
    // the mass that left through this wall in the last streaming: the
    // populations of the column's first three nodes that point out of the
    // domain (their slots are pulled by no node)
    double out = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const int k = SIDE == 0 ? d : nm - 1 - d;
        const int cell = k * p.nlayer + cil;
#pragma unroll
        for (int j = 0; j < L::Q; ++j)
            if (SIDE == 0 ? cnorm<L>(j) < -d : cnorm<L>(j) > d) out += stored_population<L, ST, FM>(p, fin, j, cell, k);
    }
    const double want = out - p.mflu[(long long)(2 * SIDE) * p.nlayer + cil] -
                        p.mflu[(long long)(2 * SIDE + 1) * p.nlayer + cil];
    // the reflection of the first fluid node's previous-step fields
    const int s1 = wall_slot(SIDE == 0 ? 1 : nm - 2, nm);
    const double* t1 = tgt_in + (long long)s1 * (D + 2) * p.nlayer + cil;
    double udes[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int a = 0; a < D; ++a) udes[a] = 2.0 * (double)p.uwall[SIDE][a] - t1[(long long)(1 + a) * p.nlayer];
    const bool iso = p.flags & KF_ISO;
    const double thdes = iso ? 1.0 : 2.0 * (double)p.twall[SIDE] - t1[(long long)(1 + D) * p.nlayer];
    // start from the target of the previous step
    const double* tw = tgt_in + (long long)warm_slot(SIDE) * (D + 2) * p.nlayer + cil;
    WallState T;
    T.rho = tw[0];
    T.u[0] = T.u[1] = T.u[2] = 0.0;
#pragma unroll
    for (int a = 0; a < D; ++a) T.u[a] = tw[(long long)(1 + a) * p.nlayer];
    T.theta = tw[(long long)(1 + D) * p.nlayer];
    // and with the Jacobian factors of the previous step, if there are any
    double LU[4][4];
    const double* lu = tgt_in + tgt_lu_offset(D, SIDE, p.nlayer) + cil;
#pragma unroll
    for (int k = 0; k < 16; ++k) LU[k / 4][k % 4] = lu[(long long)k * p.nlayer];
    const bool have = LU[0][0] != 0.0;
    const bool ok = iso ? wall_solve<L, SIDE, D>(p, fo, f, K, want, udes, thdes, T, LU, have)
                        : wall_solve<L, SIDE, D + 1>(p, fo, f, K, want, udes, thdes, T, LU, have);
    if (!ok) raise_err(p, HOLB_ERR_WALL_BIT);
    double* ws = p.wsol + (long long)SIDE * WSOL_COMPS * p.nlayer + cil;
    ws[0] = T.rho;
    ws[p.nlayer] = T.u[0];
    ws[2 * (long long)p.nlayer] = T.u[1];
    ws[3 * (long long)p.nlayer] = T.u[2];
    ws[4 * (long long)p.nlayer] = T.theta;
#pragma unroll
    for (int k = 0; k < 16; ++k) ws[(long long)(5 + k) * p.nlayer] = LU[k / 4][k % 4];
    // the wall node closed at the solved target, for every pass
    WallState after;
    wall_close<L, SIDE, true>(p, fo, f, K, T, after);
    store_closed<L, SIDE>(p, 0, cil, f);
    if (theta_out) theta_out[k0 * p.nlayer + cil] = theta_field64(p, after);
}

template <class L, int ST, int FM>
__global__ void __launch_bounds__(64)
k_wall_solve(const KParams p, const typename Codec<ST>::T* __restrict__ fin, const double* __restrict__ tgt_in,
             float* __restrict__ theta_out)
{
    const int cil = blockIdx.x * 64 + threadIdx.x;
    if (cil >= p.nlayer) return;
    if (blockIdx.y == 0) wall_solve_cell<L, ST, FM, 0>(p, fin, tgt_in, theta_out, cil);
    else wall_solve_cell<L, ST, FM, 1>(p, fin, tgt_in, theta_out, cil);
}

template <class L, int ST, int FAM, bool WALLS, int FM>
__global__ void __launch_bounds__(GEN_BLOCK)
k_aux(const KParams p, const PlaneSet ps, const typename Codec<ST>::T* __restrict__ fin,
      const double* __restrict__ tgt_in, float* __restrict__ aux_f, double* __restrict__ aux_d, int remap)
{
    const int c = xcd_block(remap) * GEN_BLOCK + threadIdx.x;
    if (c >= (ps.n0 + ps.n1) * p.nlayer) return;
    if (FM != FM_PLANE && (p.flags & KF_ISO))
        aux_cell<L, ST, FAM, WALLS, FM, true>(p, fin, tgt_in, aux_f, aux_d, plane_cell(p, ps, c));
    else
        aux_cell<L, ST, FAM, WALLS, FM>(p, fin, tgt_in, aux_f, aux_d, plane_cell(p, ps, c));
}

template <class L, int ST, int FAM, bool WALLS, int FM>
__global__ void __launch_bounds__(GEN_BLOCK)
k_step(const KParams p, const PlaneSet ps, const typename Codec<ST>::T* __restrict__ fin,
       typename Codec<ST>::T* __restrict__ fout, const float* __restrict__ aux_f, const double* __restrict__ aux_d,
       const double* __restrict__ tgt_in, double* __restrict__ tgt_out, float* __restrict__ theta_out, int remap)
{
    const int c = xcd_block(remap) * GEN_BLOCK + threadIdx.x;
    if (c >= (ps.n0 + ps.n1) * p.nlayer) return;
    // per-cell frames of an isothermal run: the shorter frame decode
    if (FM != FM_PLANE && (p.flags & KF_ISO))
        step_cell<L, ST, FAM, WALLS, FM, true>(p, fin, fout, aux_f, aux_d, tgt_in, tgt_out, plane_cell(p, ps, c),
                                               theta_out);
    else
        step_cell<L, ST, FAM, WALLS, FM>(p, fin, fout, aux_f, aux_d, tgt_in, tgt_out, plane_cell(p, ps, c),
                                         theta_out);
}

template <class L, int ST, int FAM, bool WALLS, int FM>
__global__ void __launch_bounds__(GEN_BLOCK)
k_fields(const KParams p, const typename Codec<ST>::T* __restrict__ fin, const float* __restrict__ aux_f,
         const double* __restrict__ aux_d, const double* __restrict__ tgt_in, float* __restrict__ rho_out,
         float* __restrict__ u_out, float* __restrict__ th_out)
{
    const int cell = xcd_block() * GEN_BLOCK + threadIdx.x;
    if (cell >= p.N) return;
    int x, y, z;
    cell_coords<L>(p, cell, x, y, z);
    float f[L::Q], dr, j[3], ed;
    Frame fo;
    load_state<L, ST, WALLS, FM>(p, fin, tgt_in, x, y, z, f, fo, dr, j, ed);
    Macro m;
    float pc;
    full_macro<L, ST, FAM>(p, fo, aux_f, aux_d, x, y, z, dr, j, ed, m, pc);
    if (rho_out) rho_out[cell] = m.rho;
    if (u_out) {
#pragma unroll
        for (int a = 0; a < L::D; ++a) u_out[(long long)a * p.N + cell] = m.u[a];
    }
    if (th_out) th_out[cell] = m.theta;
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Block partials of mass, momentum and energy in FP64 (wavefront shuffles,
// then LDS across the block's waves).
template <class L, int ST, int FAM, bool WALLS, int FM>
__global__ void __launch_bounds__(GEN_BLOCK)
k_reduce(const KParams p, const typename Codec<ST>::T* __restrict__ fin, const float* __restrict__ aux_f,
         const double* __restrict__ aux_d, const double* __restrict__ tgt_in, double* __restrict__ partials)
{
    __shared__ double red[GEN_BLOCK / 64][5];
    const int cell = blockIdx.x * GEN_BLOCK + threadIdx.x;
    double v[5] = {0, 0, 0, 0, 0};
    if (cell < p.N) {
        int x, y, z;
        cell_coords<L>(p, cell, x, y, z);
        float f[L::Q], dr, j[3], ed;
        Frame fo;
        load_state<L, ST, WALLS, FM>(p, fin, tgt_in, x, y, z, f, fo, dr, j, ed);
        Macro m;
        float pc;
        full_macro<L, ST, FAM>(p, fo, aux_f, aux_d, x, y, z, dr, j, ed, m, pc);
        // mass from the frame and the deviation moment, in FP64
        const double r = (double)fo.rho + (double)m.dr;
        v[0] = r;
        v[1] = r * (double)m.u[0];
        v[2] = r * (double)m.u[1];
        v[3] = r * (double)m.u[2];
        const double uu = (double)m.u[0] * m.u[0] + (double)m.u[1] * m.u[1] + (double)m.u[2] * m.u[2];
        v[4] = 0.5 * (r * uu + r * (L::D * L::c0sq) * ((1.0 + (double)fo.thb) + (double)m.dth));
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        double s = wave_sum(v[k]);
        if (lane == 0) red[wv][k] = s;
    }
    __syncthreads();
    if (threadIdx.x < 5) {
        double s = 0.0;
        for (int w = 0; w < GEN_BLOCK / 64; ++w) s += red[w][threadIdx.x];
        partials[(long long)blockIdx.x * 5 + threadIdx.x] = s;
    }
}

// Deterministic second pass: fixed strided order, then a fixed tree.
template <int UNUSED = 0>
__global__ void __launch_bounds__(256) k_reduce_final(const double* __restrict__ partials, int nblocks,
                                                      double* __restrict__ out)
{
    __shared__ double red[4][5];
    double v[5] = {0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < nblocks; b += 256)
#pragma unroll
        for (int k = 0; k < 5; ++k) v[k] += partials[(long long)b * 5 + k];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        double s = wave_sum(v[k]);
        if (lane == 0) red[wv][k] = s;
    }
    __syncthreads();
    if (threadIdx.x < 5) out[threadIdx.x] = ((red[0][threadIdx.x] + red[1][threadIdx.x]) + red[2][threadIdx.x]) +
                                           red[3][threadIdx.x];
}

// -------------------------------------------------------------- launchers

inline int nblocks_for(int N) { return (N + GEN_BLOCK - 1) / GEN_BLOCK; }

template <class L, int ST, int FAM, int FM>
struct Launch {
    using T = typename Codec<ST>::T;

    static int nm(const KParams& p) { return L::D == 3 ? p.nz : p.ny; }
    // variant 0 cell order, 1 XCD-contiguous eighths, 2 plane bands per XCD
    // (an eighth of a plane each), 3, 4, 5 bands of 4, 8, 16 blocks per XCD
    // (argument of xcd_block)
    static int remap(const LaunchCtx& c)
    {
        if (c.variant == 1) return -1;
        if (c.variant == 2) {
            const int bpp = c.kp.nlayer / GEN_BLOCK;  // blocks per plane
            return (c.kp.nlayer % GEN_BLOCK == 0 && bpp % 8 == 0) ? bpp / 8 : 0;
        }
        if (c.variant >= 3 && c.variant <= 5) return 4 << (c.variant - 3);
        return 0;
    }
    static PlaneSet all(const KParams& p) { return PlaneSet{0, nm(p), 0, 0}; }

    static hipError_t init(const LaunchCtx& c, const float* rho, const float* u, const float* th)
    {
        if constexpr (FM != FM_PLANE) {
            hipLaunchKernelGGL((k_init_frame<L, ST, FM>), dim3(nblocks_for(c.kp.N)), dim3(GEN_BLOCK), 0, c.stream,
                               c.kp, rho, u, th, (T*)c.pop_out);
        } else {
            const int n = nm(c.kp);
            hipLaunchKernelGGL(k_plane_frames<0>, dim3(n), dim3(256), 0, c.stream, c.kp, rho, th,
                               (float*)c.kp.plane_frame);
            hipError_t r = hipGetLastError();
            if (r != hipSuccess) return r;
            hipLaunchKernelGGL((k_plane_shift<L>), dim3(n), dim3(64), 0, c.stream, c.kp, c.kp.plane_frame,
                               (float*)c.kp.plane_shift);
        }
        hipError_t r = hipGetLastError();
        if (r != hipSuccess) return r;
        hipLaunchKernelGGL((k_init<L, ST, FM>), dim3(nblocks_for(c.kp.N)), dim3(GEN_BLOCK), 0, c.stream, c.kp, rho, u,
                           th, (T*)c.pop_out, c.tgt_out);
        return hipGetLastError();
    }

    // Walled domains: solve the wall-node targets of the current state
    // (before any pass that closes the wall layers).  With the thermal
    // source the same two kernels also write the temperature field of the
    // wall layers, which the field pass then skips.
    static hipError_t wall_prep(const LaunchCtx& c)
    {
        if (!c.kp.walls) return hipSuccess;
        // (not when the gradient reads the previous step's field, which
        // the collision writes)
        float* th = (FAM == FAM_THERMAL && !c.theta_out) ? c.aux_f : nullptr;
        hipLaunchKernelGGL((k_wall_fluid<L, ST, FM>), dim3(nblocks_for(4 * c.kp.nlayer)), dim3(GEN_BLOCK), 0,
                           c.stream, c.kp, (const T*)c.pop_in, c.tgt_in, th);
        hipError_t r = hipGetLastError();
        if (r != hipSuccess) return r;
        hipLaunchKernelGGL((k_wall_solve<L, ST, FM>), dim3((c.kp.nlayer + 63) / 64, 2), dim3(64), 0, c.stream, c.kp,
                           (const T*)c.pop_in, c.tgt_in, th);
        return hipGetLastError();
    }

    // walls: the planes need the TMS closure (a wall layer of a walled domain)
    static hipError_t aux_planes(const LaunchCtx& c, const PlaneSet& ps, bool walls)
    {
        if (FAM == FAM_LOCAL) return hipSuccess;
        const int n = (ps.n0 + ps.n1) * c.kp.nlayer;
        if (n == 0) return hipSuccess;
        const dim3 grid(nblocks_for(n));
        if (walls)
            hipLaunchKernelGGL((k_aux<L, ST, FAM, true, FM>), grid, dim3(GEN_BLOCK), 0, c.stream, c.kp, ps,
                               (const T*)c.pop_in, c.tgt_in, c.aux_f, c.aux_d, remap(c));
        else
            hipLaunchKernelGGL((k_aux<L, ST, FAM, false, FM>), grid, dim3(GEN_BLOCK), 0, c.stream, c.kp, ps,
                               (const T*)c.pop_in, c.tgt_in, c.aux_f, c.aux_d, remap(c));
        return hipGetLastError();
    }

    static hipError_t step_planes(const LaunchCtx& c, const PlaneSet& ps, bool walls)
    {
        const int n = (ps.n0 + ps.n1) * c.kp.nlayer;
        if (n == 0) return hipSuccess;
        const dim3 grid(nblocks_for(n));
        if (walls)
            hipLaunchKernelGGL((k_step<L, ST, FAM, true, FM>), grid, dim3(GEN_BLOCK), 0, c.stream, c.kp, ps,
                               (const T*)c.pop_in, (T*)c.pop_out, c.aux_f, c.aux_d, c.tgt_in, c.tgt_out,
                               c.theta_out, remap(c));
        else
            hipLaunchKernelGGL((k_step<L, ST, FAM, false, FM>), grid, dim3(GEN_BLOCK), 0, c.stream, c.kp, ps,
                               (const T*)c.pop_in, (T*)c.pop_out, c.aux_f, c.aux_d, c.tgt_in, c.tgt_out,
                               c.theta_out, remap(c));
        return hipGetLastError();
    }

    // Wall layers of a walled domain: the three planes next to each wall.
    static PlaneSet wall_layers(const KParams& p) { return PlaneSet{0, 3, nm(p) - 3, 3}; }
    static PlaneSet inner_planes(const KParams& p) { return PlaneSet{3, nm(p) - 6, 0, 0}; }

    // Field pass of the current state; with walls, the interior planes only
    // (wall_prep, which always runs first, has written the wall layers).
    static hipError_t aux(const LaunchCtx& c)
    {
        if (!c.kp.walls) return aux_planes(c, all(c.kp), false);
        return aux_planes(c, inner_planes(c.kp), false);
    }

    static hipError_t mark(const LaunchCtx& c, hipEvent_t e)
    {
        return e ? hipEventRecord(e, c.stream) : hipSuccess;
    }

    // The dominant launch of a step between the two timing events.
    template <class F>
    static hipError_t timed(const LaunchCtx& c, F&& launch)
    {
        hipError_t r = mark(c, c.ev_begin);
        if (r == hipSuccess) r = launch();
        if (r == hipSuccess) r = mark(c, c.ev_end);
        return r;
    }

    // A walled step on two streams.  The closure solve of the wall nodes
    // depends on the current state only, so it runs beside the work that
    // does not read it: with the same step's gradient, the field pass of the
    // interior planes (both collisions then follow on the main stream, the
    // dominant one alone); with grad_lag (the last step's field, no field
    // pass), the interior collision, the wall-layer collision following the
    // solve on the second stream.  The two streams never write the same
    // words: the wall work writes the wall layers' closures, targets, theta
    // and populations, the main stream the interior planes'.
    static hipError_t step_two_streams(const LaunchCtx& c)
    {
        LaunchCtx w = c;
        w.stream = c.side;
        w.ev_begin = w.ev_end = nullptr;
        hipError_t r = hipEventRecord(c.ev_fork, c.stream);
        if (r == hipSuccess) r = hipStreamWaitEvent(c.side, c.ev_fork, 0);
        if (r == hipSuccess) r = wall_prep(w);
        if (!c.theta_out) {
            if (r == hipSuccess) r = hipEventRecord(c.ev_wall, c.side);
            if (r == hipSuccess) r = aux(c);
            if (r == hipSuccess) r = hipStreamWaitEvent(c.stream, c.ev_wall, 0);
            if (r == hipSuccess) r = step_planes(c, wall_layers(c.kp), true);
            if (r == hipSuccess) r = timed(c, [&] { return step_planes(c, inner_planes(c.kp), false); });
            return r;
        }
        if (r == hipSuccess) r = step_planes(w, wall_layers(c.kp), true);
        if (r == hipSuccess) r = hipEventRecord(c.ev_join, c.side);
        if (r == hipSuccess) r = timed(c, [&] { return step_planes(c, inner_planes(c.kp), false); });
        if (r == hipSuccess) r = hipStreamWaitEvent(c.stream, c.ev_join, 0);
        return r;
    }

    static hipError_t step(const LaunchCtx& c)
    {
        if (c.kp.walls && c.side) return step_two_streams(c);
        hipError_t r = wall_prep(c);
        if (r == hipSuccess && !c.theta_out) r = aux(c);
        if (r != hipSuccess) return r;
        if (!c.kp.walls) return timed(c, [&] { return step_planes(c, all(c.kp), false); });
        r = step_planes(c, wall_layers(c.kp), true);
        if (r == hipSuccess) r = timed(c, [&] { return step_planes(c, inner_planes(c.kp), false); });
        return r;
    }

    static void dominant(const LaunchCtx& c, char* name, size_t len, long long* cells)
    {
        const int n = nm(c.kp);
        const int planes = c.kp.walls ? n - 6 : n;
        if (cells) *cells = (long long)planes * c.kp.nlayer;
        if (!name || !len) return;
        snprintf(name, len, "k_step<%s,%d,%d,false,%d>", L::D == 3 ? "D3Q39" : "D2Q37", ST, FAM, FM);
    }

    static hipError_t fields(const LaunchCtx& c, float* rho, float* u, float* th)
    {
        hipError_t rp = wall_prep(c);
        if (rp != hipSuccess) return rp;
        if (FAM == FAM_PTENSOR) {
            hipError_t r = aux(c);
            if (r != hipSuccess) return r;
        }
        if (c.kp.walls)
            hipLaunchKernelGGL((k_fields<L, ST, FAM, true, FM>), dim3(nblocks_for(c.kp.N)), dim3(GEN_BLOCK), 0,
                               c.stream, c.kp, (const T*)c.pop_in, c.aux_f, c.aux_d, c.tgt_in, rho, u, th);
        else
            hipLaunchKernelGGL((k_fields<L, ST, FAM, false, FM>), dim3(nblocks_for(c.kp.N)), dim3(GEN_BLOCK), 0,
                               c.stream, c.kp, (const T*)c.pop_in, c.aux_f, c.aux_d, c.tgt_in, rho, u, th);
        return hipGetLastError();
    }

    static hipError_t reduce(const LaunchCtx& c, double* out)
    {
        hipError_t rp = wall_prep(c);
        if (rp != hipSuccess) return rp;
        if (FAM == FAM_PTENSOR) {
            hipError_t r = aux(c);
            if (r != hipSuccess) return r;
        }
        const int nb = nblocks_for(c.kp.N);
        if (nb > c.max_partials) return hipErrorInvalidValue;
        if (c.kp.walls)
            hipLaunchKernelGGL((k_reduce<L, ST, FAM, true, FM>), dim3(nb), dim3(GEN_BLOCK), 0, c.stream, c.kp,
                               (const T*)c.pop_in, c.aux_f, c.aux_d, c.tgt_in, c.partials);
        else
            hipLaunchKernelGGL((k_reduce<L, ST, FAM, false, FM>), dim3(nb), dim3(GEN_BLOCK), 0, c.stream, c.kp,
                               (const T*)c.pop_in, c.aux_f, c.aux_d, c.tgt_in, c.partials);
        hipError_t r = hipGetLastError();
        if (r != hipSuccess) return r;
        hipLaunchKernelGGL(k_reduce_final<0>, dim3(1), dim3(256), 0, c.stream, c.partials, nb, out);
        return hipGetLastError();
    }
};

template <class L, int ST, int FM>
inline hipError_t dispatch_family(const LaunchCtx& c, int op, const float* a, const float* b, const float* d,
                                  float* o1, float* o2, float* o3, double* dout)
{
#define HOLB_OPS(FAM)                                                  \
    switch (op) {                                                      \
    case 0: return Launch<L, ST, FAM, FM>::init(c, a, b, d);           \
    case 1: return Launch<L, ST, FAM, FM>::step(c);                    \
    case 2: {                                                          \
        hipError_t r = Launch<L, ST, FAM, FM>::wall_prep(c);           \
        return r == hipSuccess ? Launch<L, ST, FAM, FM>::aux(c) : r;   \
    }                                                                  \
    case 3: return Launch<L, ST, FAM, FM>::fields(c, o1, o2, o3);      \
    case 4: return Launch<L, ST, FAM, FM>::reduce(c, dout);            \
    }
    switch (c.family) {
    case FAM_LOCAL: HOLB_OPS(FAM_LOCAL) break;
    case FAM_THERMAL: HOLB_OPS(FAM_THERMAL) break;
    case FAM_PTENSOR: HOLB_OPS(FAM_PTENSOR) break;
    }
#undef HOLB_OPS
    return hipErrorInvalidValue;
}

// Entry of one instantiation unit: every family and frame mode of lattice L
// for FP32 storage (SIXTEEN = false) or for the two 16-bit forms.
template <class L, bool SIXTEEN>
inline hipError_t dispatch_set(const LaunchCtx& c, int op, const float* a, const float* b, const float* d,
                               float* o1, float* o2, float* o3, double* dout)
{
    if constexpr (!SIXTEEN) {
        // per-plane frames are FP32 only (validated on the host)
        if (c.frames == FM_PLANE) return dispatch_family<L, ST_F32, FM_PLANE>(c, op, a, b, d, o1, o2, o3, dout);
        return dispatch_family<L, ST_F32, FM_CELL>(c, op, a, b, d, o1, o2, o3, dout);
    } else {
        if (c.frames == FM_PLANE) {
            if (c.storage == ST_F16) return dispatch_family<L, ST_F16, FM_PLANE>(c, op, a, b, d, o1, o2, o3, dout);
            return dispatch_family<L, ST_BF16, FM_PLANE>(c, op, a, b, d, o1, o2, o3, dout);
        }
        if (c.frames == FM_CELLU) {
            if (c.storage == ST_F16) return dispatch_family<L, ST_F16, FM_CELLU>(c, op, a, b, d, o1, o2, o3, dout);
            return dispatch_family<L, ST_BF16, FM_CELLU>(c, op, a, b, d, o1, o2, o3, dout);
        }
        if (c.storage == ST_F16) return dispatch_family<L, ST_F16, FM_CELL>(c, op, a, b, d, o1, o2, o3, dout);
        return dispatch_family<L, ST_BF16, FM_CELL>(c, op, a, b, d, o1, o2, o3, dout);
    }
}

#define HOLB_DISPATCH_ARGS \
    const LaunchCtx &c, int op, const float *a, const float *b, const float *d, float *o1, float *o2, float *o3, \
        double *dout
hipError_t dispatch_d2_f32(HOLB_DISPATCH_ARGS);
hipError_t dispatch_d2_16(HOLB_DISPATCH_ARGS);
hipError_t dispatch_d3_f32(HOLB_DISPATCH_ARGS);
hipError_t dispatch_d3_16(HOLB_DISPATCH_ARGS);

}  // namespace holb
