// Device-side building blocks of the fused high-order LBM step (gfx950).
//
// Every kernel variant (generic one-cell-per-thread, plane-marching, batched)
// calls the same inline functions below, and the library is compiled with
// -ffp-contract=off and explicit fmaf(), so the per-cell arithmetic -- and
// therefore the result -- is bitwise identical across tilings.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "holb_params.h"
#include "lattice_tables.h"

namespace holb {

// ---------------------------------------------------------------- lattice

template <class L>
struct Lat : L {
    static constexpr float w(int i) { return (float)L::shell_w[L::shell[i]]; }
    static constexpr float invw(int i) { return (float)(1.0 / L::shell_w[L::shell[i]]); }
    static constexpr int c2(int i) { return L::cx[i] * L::cx[i] + L::cy[i] * L::cy[i] + L::cz[i] * L::cz[i]; }
    static constexpr float ic0sq = (float)(1.0 / L::c0sq);
    static constexpr float c0sq_f = (float)L::c0sq;
    // opposite index: rest is 0, pairs are (1+2p, 2+2p)
    static constexpr int opp(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }
    // velocity component along the wall-normal (last) axis
    static constexpr int cw(int i) { return L::D == 2 ? L::cy[i] : L::cz[i]; }
};

// ------------------------------------------------------------------ codec
// 16-bit storage holds q = f / w - r, r = f^eq_i(reference) / w_i, rounded to
// nearest-even; decoding is f = w (r + q).

template <int ST>
struct Codec;

template <>
struct Codec<ST_F32> {
    using T = float;
    static __device__ __forceinline__ float dec(T v, float, float) { return v; }
    static __device__ __forceinline__ T enc(float f, float, float) { return f; }
};

template <>
struct Codec<ST_F16> {
    using T = uint16_t;
    static __device__ __forceinline__ float dec(T v, float w, float r)
    {
        return w * (r + (float)__builtin_bit_cast(_Float16, v));
    }
    static __device__ __forceinline__ T enc(float f, float invw, float r)
    {
        return __builtin_bit_cast(uint16_t, (_Float16)(f * invw - r));
    }
};

__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);  // quiet NaN
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

template <>
struct Codec<ST_BF16> {
    using T = uint16_t;
    static __device__ __forceinline__ float dec(T v, float w, float r)
    {
        return w * (r + __uint_as_float((uint32_t)v << 16));
    }
    static __device__ __forceinline__ T enc(float f, float invw, float r)
    {
        return f32_to_bf16_rne(f * invw - r);
    }
};

// -------------------------------------------------------- small helpers

__device__ __forceinline__ int wrapc(int v, int n)
{
    while (v < 0) v += n;
    while (v >= n) v -= n;
    return v;
}

__device__ __forceinline__ void raise_err(const KParams& p, unsigned bit)
{
    if (p.err) atomicOr(p.err, bit);
}

// ----------------------------------------------------- kinetic algebra
// Lattice units outside; a = c.u / c0^2, uu = |u|^2 / c0^2, xx = |c|^2 / c0^2
// are the Hermite-scaled invariants of Eq. (2.2) and Table 2.

// Eq. (2.2) for one direction (used by the wall closure and the
// initialisation; the collision evaluates it per +/-c pair instead).
template <class L>
__device__ __forceinline__ float feq_one(int i, float rho, const float (&u)[3], float theta)
{
    using LL = Lat<L>;
    constexpr float D = (float)L::D;
    const float ic = LL::ic0sq;
    float a = ((float)L::cx[i] * u[0] + (float)L::cy[i] * u[1] + (float)L::cz[i] * u[2]) * ic;
    float uu = (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]) * ic;
    float xx = (float)LL::c2(i) * ic;
    float thb = theta - 1.0f;
    float a2 = a * a;
    float t = 1.0f + a + 0.5f * a2 - 0.5f * uu + 0.5f * thb * (xx - D)
            + a2 * a * (1.0f / 6.0f) - 0.5f * a * uu + 0.5f * a * thb * (xx - (D + 2.0f))
            + a2 * a2 * (1.0f / 24.0f) - 0.25f * a2 * uu + 0.125f * uu * uu
            + 0.25f * thb * (a2 * (xx - (D + 4.0f)) + uu * ((D + 2.0f) - xx))
            + 0.125f * thb * thb * (xx * xx - 2.0f * (D + 2.0f) * xx + D * (D + 2.0f));
    return LL::w(i) * rho * t;
}

// Shifted moments of Eq. (4.5): rho = sum f, rho u = sum c f + F/2, and
// rho D c0^2 theta = sum |c|^2 f - rho |u|^2 + u.F (tr G_2 = 2 u.F).
struct Macro {
    float rho, u[3], theta, F[3];
};

template <class L>
__device__ __forceinline__ void moments(const float (&f)[L::Q], float& rho, float (&j)[3], float& e)
{
    using LL = Lat<L>;
    rho = 0.f;
    j[0] = j[1] = j[2] = 0.f;
    e = 0.f;
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        rho += f[i];
        if (L::cx[i]) j[0] = fmaf((float)L::cx[i], f[i], j[0]);
        if (L::cy[i]) j[1] = fmaf((float)L::cy[i], f[i], j[1]);
        if (L::cz[i]) j[2] = fmaf((float)L::cz[i], f[i], j[2]);
        if (LL::c2(i)) e = fmaf((float)LL::c2(i), f[i], e);
    }
}

template <class L>
__device__ __forceinline__ void macro_from_moments(const KParams& p, float rho, const float (&j)[3], float e,
                                                   const float (&Fext)[3], Macro& m)
{
    constexpr float DC = (float)(L::D * L::c0sq);
    m.rho = rho;
    const bool body = p.flags & KF_BODY;
    float ir = 1.0f / rho;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        float F = (body && a < L::D) ? rho * p.g[a] : 0.0f;
        F += Fext[a];
        m.F[a] = F;
        m.u[a] = (j[a] + 0.5f * F) * ir;
    }
    if (p.flags & KF_ISO) {
        m.theta = 1.0f;
    } else {
        float uu = m.u[0] * m.u[0] + m.u[1] * m.u[1] + m.u[2] * m.u[2];
        float uF = m.u[0] * m.F[0] + m.u[1] * m.F[1] + m.u[2] * m.F[2];
        m.theta = (e - rho * uu + uF) / (rho * DC);
    }
    if (!(rho > 0.0f) || !(rho < 3.0e38f)) raise_err(p, HOLB_ERR_DENSITY_BIT);
    if (!(m.theta > 0.0f) || !(m.theta < 3.0e38f)) raise_err(p, HOLB_ERR_THETA_BIT);
}

// Section 4.3, Eqs. (4.7)-(4.8): rebuild the populations that streamed in
// from outside the walls.  unk has bit i set for unknown direction i; tgt
// holds the previous-step (rho, u[D], theta) of this node; wall = 0/1 for a
// wall node (first/last layer), -1 for a fluid node.
template <class L>
__device__ __forceinline__ void tms_fill(const KParams& p, float (&f)[L::Q], uint64_t unk, int wall,
                                         const float* tgt)
{
    using LL = Lat<L>;
    constexpr int D = L::D;
    float rt = tgt[0];
    float ut[3] = {0.f, 0.f, 0.f};
    float tt;
    if (wall >= 0) {
#pragma unroll
        for (int a = 0; a < D; ++a) ut[a] = p.uwall[wall][a];
        tt = p.twall[wall];
    } else {
#pragma unroll
        for (int a = 0; a < D; ++a) ut[a] = tgt[1 + a];
        tt = tgt[1 + D];
    }
    if (p.flags & KF_ISO) tt = 1.0f;
    float rl = 0.f, jl[3] = {0.f, 0.f, 0.f}, el = 0.f;
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        if ((unk >> i) & 1ull) f[i] = feq_one<L>(i, rt, ut, tt);  // target equilibrium, for now
        rl += f[i];
        if (L::cx[i]) jl[0] = fmaf((float)L::cx[i], f[i], jl[0]);
        if (L::cy[i]) jl[1] = fmaf((float)L::cy[i], f[i], jl[1]);
        if (L::cz[i]) jl[2] = fmaf((float)L::cz[i], f[i], jl[2]);
        if (LL::c2(i)) el = fmaf((float)LL::c2(i), f[i], el);
    }
    const float zero3[3] = {0.f, 0.f, 0.f};
    Macro loc;
    KParams q = p;
    q.err = nullptr;
    macro_from_moments<L>(q, rl, jl, el, zero3, loc);
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        if ((unk >> i) & 1ull) f[i] = f[LL::opp(i)] + f[i] - feq_one<L>(i, loc.rho, loc.u, loc.theta);
    }
}

// Eq. (4.4) collision with f^eq of Eq. (2.2) and S = F (Eq. 3.3) + H (Eq. 3.7)
// + P (Eq. 3.12), evaluated once per +/-c pair from its even and odd parts.
//   hc    = (1 - 1/Pr) rho theta / 2   (0 without the thermal source)
//   gT    = grad theta per lattice spacing
//   pc    = -(k / (2 D tau)) |F^SC|^2 / (c0^2 G psi^2)   (0 without it)
template <class L>
__device__ __forceinline__ void collide(const KParams& p, float (&f)[L::Q], const Macro& m, float hc,
                                        const float (&gT)[3], float pc)
{
    using LL = Lat<L>;
    constexpr int D = L::D;
    constexpr float Df = (float)D;
    const float ic = LL::ic0sq;
    const float uu = (m.u[0] * m.u[0] + m.u[1] * m.u[1] + m.u[2] * m.u[2]) * ic;
    const float UF = (m.u[0] * m.F[0] + m.u[1] * m.F[1] + m.u[2] * m.F[2]) * ic;
    const float thb = m.theta - 1.0f;
    const float om = p.omega, ka = p.kappa, om1 = 1.0f - p.omega;
    const float orho = om * m.rho;
    const float U[3] = {m.u[0] * ic, m.u[1] * ic, m.u[2] * ic};
    const float Ph[3] = {m.F[0] * ic, m.F[1] * ic, m.F[2] * ic};

    float K0[L::NS], K1[L::NS], K2[L::NS], M1[L::NS], HS[L::NS], PS[L::NS];
    const float c_uu = 1.0f - 0.5f * uu;
#pragma unroll
    for (int s = 0; s < L::NS; ++s) {
        const float xx = (float)L::shell_c2[s] * ic;
        const float q2 = 0.125f * (xx * xx - 2.0f * (Df + 2.0f) * xx + Df * (Df + 2.0f));
        K0[s] = c_uu + 0.125f * uu * uu + thb * (0.5f * (xx - Df) + 0.25f * uu * ((Df + 2.0f) - xx) + thb * q2);
        K1[s] = c_uu + 0.5f * thb * (xx - Df - 2.0f);
        K2[s] = 0.5f - 0.25f * uu + 0.25f * thb * (xx - Df - 4.0f);
        M1[s] = 1.0f + 0.5f * (thb * (xx - Df - 2.0f) - uu);
        HS[s] = hc * (xx - Df - 2.0f);
        PS[s] = pc * (xx - Df);
    }
    // rest velocity
    f[0] = fmaf(om1, f[0], LL::w(0) * fmaf(orho, K0[0], ka * (PS[0] - UF)));
#pragma unroll
    for (int pp = 0; pp < L::NP; ++pp) {
        const int i = 1 + 2 * pp;
        const int s = L::shell[i];
        constexpr float sixth = 1.0f / 6.0f, c24 = 1.0f / 24.0f;
        float a = 0.f, b = 0.f, h = 0.f;
        if (L::cx[i]) { a = fmaf((float)L::cx[i], U[0], a); b = fmaf((float)L::cx[i], Ph[0], b); h = fmaf((float)L::cx[i], gT[0], h); }
        if (L::cy[i]) { a = fmaf((float)L::cy[i], U[1], a); b = fmaf((float)L::cy[i], Ph[1], b); h = fmaf((float)L::cy[i], gT[1], h); }
        if (L::cz[i]) { a = fmaf((float)L::cz[i], U[2], a); b = fmaf((float)L::cz[i], Ph[2], b); h = fmaf((float)L::cz[i], gT[2], h); }
        const float a2 = a * a;
        const float fe = fmaf(a2, fmaf(a2, c24, K2[s]), K0[s]);
        const float fo = a * fmaf(a2, sixth, K1[s]);
        const float se = fmaf(a, b, PS[s] - UF);
        const float so = fmaf(b, fmaf(0.5f, a2, M1[s]), fmaf(HS[s], h, -a * UF));
        const float E = fmaf(orho, fe, ka * se);
        const float O = fmaf(orho, fo, ka * so);
        const float w = LL::w(i);
        f[i] = fmaf(om1, f[i], w * (E + O));
        f[i + 1] = fmaf(om1, f[i + 1], w * (E - O));
    }
}

// van der Waals pseudopotential of Eq. (3.8) in FP64:
// psi = sqrt(2 (p_EOS - rho c0^2) / (G c0^2)).
__device__ __forceinline__ double psi_vdw(const KParams& p, double rho, double c0sq, bool& bad)
{
    double br = p.eos_b * rho;
    if (!(rho > 0.0) || !(br < 1.0)) { bad = true; return 0.0; }
    double pe = rho * p.eos_T / (1.0 - br) - p.eos_a * rho * rho;
    double arg = 2.0 * (pe - rho * c0sq) / (p.G * c0sq);
    if (!(arg >= 0.0)) { bad = true; return 0.0; }
    return sqrt(arg);
}

}  // namespace holb
