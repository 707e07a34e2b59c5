// Device-side building blocks of the fused high-order LBM step (gfx950).
//
// Populations are handled in deviation form relative to a per-cell frame: a
// node whose frame is (rho_F, theta_F) holds h_i = f_i / w_i - R_i(F), with
// R_i(F) = rho_F (1 + t_i(u = 0, theta_F)) the equilibrium bracket of Eq.
// (2.2) at rest in that frame.  Every node stores its frame (rho and theta
// rounded to binary16) beside its populations; a node that pulls population
// i from x - c_i moves it from the source's frame into its own by adding
// R_i(source) - R_i(own), formed as a difference of neighbouring values.  In
// exact arithmetic this is the same scheme; in FP32 and in 16-bit storage the
// values handled stay at the size of the local non-equilibrium and gradient
// parts instead of the variation of density and temperature across the
// domain, so their round-off is correspondingly smaller.
//
// Every kernel variant (the block orders of the generic kernels, the batched
// form) calls the same inline functions below, and the library is compiled with
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
    // D c0^2 (the energy moment of the rest state per unit density)
    static constexpr float DC = (float)(L::D * L::c0sq);
    // index of the +e_a velocity (first member of the axis pair of shell 1)
    static constexpr int axis_plus(int a)
    {
        for (int i = 1; i < L::Q; i += 2)
            if ((a == 0 ? L::cx[i] : a == 1 ? L::cy[i] : L::cz[i]) == 1 && c2(i) == 1) return i;
        return -1;
    }
    // opposite index: rest is 0, pairs are (1+2p, 2+2p)
    static constexpr int opp(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }
};

// ------------------------------------------------------------------ codec
// FP32 storage holds h_i.  16-bit storage holds q_i = h_i - d_i rounded to
// nearest-even, where d_i = (f^eq_i(rho0, u0, theta0) - f^eq_i(rho0, 0,
// theta0)) / w_i removes the bracket of a uniform background velocity u0.

template <int ST>
struct Codec;

template <>
struct Codec<ST_F32> {
    using T = float;
    static __device__ __forceinline__ float dec(T v, float) { return v; }
    static __device__ __forceinline__ T enc(float h, float) { return h; }
};

template <>
struct Codec<ST_F16> {
    using T = uint16_t;
    static __device__ __forceinline__ float dec(T v, float d) { return (float)__builtin_bit_cast(_Float16, v) + d; }
    static __device__ __forceinline__ T enc(float h, float d) { return __builtin_bit_cast(uint16_t, (_Float16)(h - d)); }
};

template <>
struct Codec<ST_BF16> {
    using T = uint16_t;
    static __device__ __forceinline__ float dec(T v, float d) { return __uint_as_float((uint32_t)v << 16) + d; }
    // hardware conversion (round to nearest even, NaN kept quiet)
    static __device__ __forceinline__ T enc(float h, float d) { return __builtin_bit_cast(uint16_t, (__bf16)(h - d)); }
};

// -------------------------------------------------------- small helpers

// Periodic wrap of a coordinate.  The stencils reach at most 3 cells past
// an edge, so one correction each way suffices on axes of 3 cells or more;
// the loop runs only on shorter axes (a branch the waves of larger domains
// skip: written as a bare loop, the wrap costs about 20 VALU per call).
__device__ __forceinline__ int wrapc(int v, int n)
{
    v = v < 0 ? v + n : v;
    v = v >= n ? v - n : v;
    if ((unsigned)v >= (unsigned)n) {
        while (v < 0) v += n;
        while (v >= n) v -= n;
    }
    return v;
}

// The same wrap as bare loops, for sequences of dependent loads on edge
// waves only: the loops keep each address next to its load, where the
// branch-free form lets the compiler compute every address of the sequence
// ahead and hold them all in registers (costing a wave of occupancy in the
// momentum phase of the per-cell momentum frames).
__device__ __forceinline__ int wrap_seq(int v, int n)
{
    while (v < 0) v += n;
    while (v >= n) v -= n;
    return v;
}

__device__ __forceinline__ void raise_err(const KParams& p, unsigned bit)
{
    if (p.err) atomicOr(p.err, bit);
}

// ------------------------------------------------------------- frames
// A node's frame: rho_F and thb_F = theta_F - 1, decoded from the packed
// binary16 pair (rho, theta - 1) stored per cell.

struct Frame {
    float rho, thb;
};

__device__ __forceinline__ uint32_t pack_frame(float rho, float thb)
{
    const uint16_t r = __builtin_bit_cast(uint16_t, (_Float16)rho);
    const uint16_t t = __builtin_bit_cast(uint16_t, (_Float16)thb);
    return (uint32_t)r | ((uint32_t)t << 16);
}

__device__ __forceinline__ Frame unpack_frame(uint32_t v)
{
    Frame F;
    F.rho = (float)__builtin_bit_cast(_Float16, (uint16_t)(v & 0xffffu));
    F.thb = (float)__builtin_bit_cast(_Float16, (uint16_t)(v >> 16));
    return F;
}

// FM_CELLU adds the first-order part of the frame bracket, c_i . P with
// P = rho_F (u_F - u0) / c0^2, so that 16-bit storage keeps the momentum part
// of the populations out of the stored deviation too.  P is carried as three
// 10-bit signed multiples of 2^-10 (|P| < 0.5; larger values saturate, which
// only makes the frame less close, never inexact) in a momentum plane after
// the frame plane; c_i . P is then an exact integer dot product times 2^-10
// on both sides.
constexpr float PSTEP = 1.0f / 1024.0f;

__device__ __forceinline__ uint32_t pack_mom(const float (&P)[3])
{
    uint32_t w = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int q = (int)fminf(fmaxf(rintf(P[a] * 1024.0f), -511.0f), 511.0f);
        w |= ((uint32_t)q & 0x3ffu) << (10 * a);
    }
    return w;
}

// c_i . P of a packed momentum word (exact).
template <class L>
__device__ __forceinline__ float cdot_mom(int i, uint32_t w)
{
    int d = 0;
    if (L::cx[i]) d += L::cx[i] * __builtin_amdgcn_sbfe((int)w, 0u, 10u);
    if (L::cy[i]) d += L::cy[i] * __builtin_amdgcn_sbfe((int)w, 10u, 10u);
    if (L::cz[i]) d += L::cz[i] * __builtin_amdgcn_sbfe((int)w, 20u, 10u);
    return (float)d * PSTEP;
}

// Per-cell frame plane stored after the Q population planes of a buffer.
template <int ST>
__device__ __forceinline__ const uint32_t* frame_plane(const void* pop, long long pitch, int Q)
{
    using T = typename Codec<ST>::T;
    return (const uint32_t*)((const T*)pop + (long long)Q * pitch);
}
template <int ST>
__device__ __forceinline__ uint32_t* frame_plane(void* pop, long long pitch, int Q)
{
    using T = typename Codec<ST>::T;
    return (uint32_t*)((T*)pop + (long long)Q * pitch);
}

// Momentum plane (FM_CELLU): one word per cell after the frame plane, which
// is padded to 256 bytes.
__device__ __forceinline__ long long mom_offset(int N) { return ((long long)N + 63) & ~63ll; }

// ----------------------------------------------------- kinetic algebra
// Lattice units outside; a = c.u / c0^2, uu = |u|^2 / c0^2, xx = |c|^2 / c0^2
// and thb = theta - 1 are the Hermite-scaled invariants of Eq. (2.2) / Table 2.

// Eq. (2.2) for one direction, minus its leading 1: f^eq_i = w_i rho (1 + t).
template <class L, class R>
__device__ __forceinline__ R feq_poly(int i, const R (&u)[3], R thb)
{
    using LL = Lat<L>;
    constexpr R D = (R)L::D;
    const R ic = (R)(1.0 / L::c0sq);
    const R a = ((R)L::cx[i] * u[0] + (R)L::cy[i] * u[1] + (R)L::cz[i] * u[2]) * ic;
    const R uu = (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]) * ic;
    const R xx = (R)LL::c2(i) * ic;
    const R a2 = a * a;
    return a + (R)0.5 * a2 - (R)0.5 * uu + (R)0.5 * thb * (xx - D)
         + a2 * a * ((R)1 / (R)6) - (R)0.5 * a * uu + (R)0.5 * a * thb * (xx - (D + (R)2))
         + a2 * a2 * ((R)1 / (R)24) - (R)0.25 * a2 * uu + (R)0.125 * uu * uu
         + (R)0.25 * thb * (a2 * (xx - (D + (R)4)) + uu * ((D + (R)2) - xx))
         + (R)0.125 * thb * thb * (xx * xx - (R)2 * (D + (R)2) * xx + D * (D + (R)2));
}

template <class L, class R = float>
__device__ __forceinline__ R feq_t(int i, const float (&uf)[3], float thbf)
{
    const R u[3] = {(R)uf[0], (R)uf[1], (R)uf[2]};
    return feq_poly<L, R>(i, u, (R)thbf);
}

// t0 = t(u = 0, theta0) for a shell of squared speed xx (in c0^2 units).
template <class L>
__device__ __forceinline__ float ref_t0(float xx, float thb0)
{
    constexpr float D = (float)L::D;
    const float q2 = 0.125f * (xx * xx - 2.0f * (D + 2.0f) * xx + D * (D + 2.0f));
    return thb0 * fmaf(thb0, q2, 0.5f * (xx - D));
}

// Frame shifts R_i(S) - R_i(O), R_i(F) = rho_F (1 + t0(thb_F)).  With
// a = rho_S - rho_O, b = thb_S - thb_O, X = xx - D and Y/8 = q2 the theta^2
// coefficient of t0, the difference of two close brackets is
//   R_i(S) - R_i(O) = a T_O + rho_S b (K_O + b q2),
//   T_O = 1 + t0(thb_O),  K_O = X/2 + 2 thb_O q2,
// formed without either bracket.  FrameRef holds T_O and K_O per shell.
template <class L>
struct FrameRef {
    float rho, thb;
    float T[L::NS], K[L::NS];
};

template <class L>
__device__ __forceinline__ float shell_q2(int s)
{
    constexpr float D = (float)L::D;
    const float xx = (float)L::shell_c2[s] * Lat<L>::ic0sq;
    return 0.125f * (xx * xx - 2.0f * (D + 2.0f) * xx + D * (D + 2.0f));
}

template <class L>
__device__ __forceinline__ float shell_hx(int s)
{
    return 0.5f * ((float)L::shell_c2[s] * Lat<L>::ic0sq - (float)L::D);
}

template <class L>
__device__ __forceinline__ FrameRef<L> frame_ref(const Frame& O)
{
    FrameRef<L> r;
    r.rho = O.rho;
    r.thb = O.thb;
#pragma unroll
    for (int s = 0; s < L::NS; ++s) {
        const float q2 = shell_q2<L>(s), hx = shell_hx<L>(s);
        r.T[s] = 1.0f + O.thb * fmaf(O.thb, q2, hx);
        r.K[s] = fmaf(2.0f * O.thb, q2, hx);
    }
    return r;
}

template <class L>
__device__ __forceinline__ float frame_shift(const FrameRef<L>& O, int s, const Frame& S)
{
    const float a = S.rho - O.rho, b = S.thb - O.thb;
    const float k = fmaf(b, shell_q2<L>(s), O.K[s]);
    return fmaf(S.rho * b, k, a * O.T[s]);
}

// f^eq_i / w_i - R_i(F) (used by the wall closure and the initialisation;
// the collision evaluates the equilibrium per +/-c pair instead).
template <class L>
__device__ __forceinline__ float feq_dev(const Frame& F, int i, float rho, const float (&u)[3], float thb)
{
    using LL = Lat<L>;
    const float t0 = ref_t0<L>((float)LL::c2(i) * LL::ic0sq, F.thb);
    return (rho - F.rho) * (1.0f + t0) + rho * (feq_t<L>(i, u, thb) - t0);
}

// Macroscopic state of a node from the shifted moments of Eq. (4.5):
// rho = sum f, rho u = sum c f + F/2, and rho D c0^2 theta = sum |c|^2 f -
// rho |u|^2 + u.F (tr G_2 = 2 u.F).  In the node's frame F: dr = rho - rho_F,
// dth = theta - theta_F, thb = theta - 1; j = sum c f and ed = sum |c|^2 f -
// rho_F D c0^2 theta_F are kept for the conservation check.
struct Macro {
    float rho, dr, u[3], dth, thb, theta, F[3];
    float j[3], ed;
};

// Deviation moments from the +/-c pairs: the pair sum carries mass and
// energy, the pair difference momentum (a difference of two close values is
// exact, so slow flows keep their full precision).
template <class L>
__device__ __forceinline__ void moments(const float (&h)[L::Q], float& dr, float (&j)[3], float& ed)
{
    using LL = Lat<L>;
    dr = LL::w(0) * h[0];
    j[0] = j[1] = j[2] = 0.f;
    ed = 0.f;
#pragma unroll
    for (int pp = 0; pp < L::NP; ++pp) {
        const int i = 1 + 2 * pp;
        const float sm = LL::w(i) * (h[i] + h[i + 1]);
        const float df = LL::w(i) * (h[i] - h[i + 1]);
        dr += sm;
        ed = fmaf((float)LL::c2(i), sm, ed);
        if (L::cx[i]) j[0] = fmaf((float)L::cx[i], df, j[0]);
        if (L::cy[i]) j[1] = fmaf((float)L::cy[i], df, j[1]);
        if (L::cz[i]) j[2] = fmaf((float)L::cz[i], df, j[2]);
    }
}

template <class L, bool RAISE = true>
__device__ __forceinline__ void macro_from_moments(const KParams& p, const Frame& fr, float dr, const float (&j)[3],
                                                   float ed, const float (&Fext)[3], Macro& m)
{
    using LL = Lat<L>;
    const float rho = fr.rho + dr;
    m.rho = rho;
    m.dr = dr;
    m.ed = ed;
    m.j[0] = j[0]; m.j[1] = j[1]; m.j[2] = j[2];
    const bool body = p.flags & KF_BODY;
    const float ir = 1.0f / rho;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        float F = (body && a < L::D) ? rho * p.g[a] : 0.0f;
        F += Fext[a];
        m.F[a] = F;
        m.u[a] = (j[a] + 0.5f * F) * ir;
    }
    if (p.flags & KF_ISO) {
        m.dth = 0.0f;
        m.thb = 0.0f;
        m.theta = 1.0f;
    } else {
        const float uu = m.u[0] * m.u[0] + m.u[1] * m.u[1] + m.u[2] * m.u[2];
        const float uF = m.u[0] * m.F[0] + m.u[1] * m.F[1] + m.u[2] * m.F[2];
        // theta - theta_F = (e - rho |u|^2 + u.F - rho D c0^2 theta_F) / (rho D c0^2)
        const float th0 = 1.0f + fr.thb;
        m.dth = ((ed - dr * (LL::DC * th0)) - rho * uu + uF) / (rho * LL::DC);
        m.thb = fr.thb + m.dth;
        m.theta = th0 + m.dth;
    }
    if (RAISE) {
        if (!(rho > 0.0f) || !(rho < 3.0e38f)) raise_err(p, HOLB_ERR_DENSITY_BIT);
        if (!(m.theta > 0.0f) || !(m.theta < 3.0e38f)) raise_err(p, HOLB_ERR_THETA_BIT);
    }
}

// FP32 compensation of the collision invariants.  In exact arithmetic the
// collision of Eq. (4.4) maps the moments (rho, j, e) to (rho, j + F,
// e + 2 u.F) (Eqs. 2.3 and 4.5); with FP32-rounded weights and coefficients
// the computed post-collision moments miss these by a small systematic
// amount that would accumulate over many steps.  The residual is put back on
// the rest population and the +/-e_a axis pairs (|c| = 1), which changes the
// result only at rounding level.  The energy target applies only when theta
// is evolved.
template <class L>
__device__ __forceinline__ void conserve(const KParams& p, float (&h)[L::Q], const Macro& m)
{
    using LL = Lat<L>;
    constexpr int D = L::D;
    float dr2, j2[3], e2;
    moments<L>(h, dr2, j2, e2);
    const float ddr = m.dr - dr2;
    float de = 0.0f;
    if (!(p.flags & KF_ISO)) {
        const float uF = m.u[0] * m.F[0] + m.u[1] * m.F[1] + m.u[2] * m.F[2];
        de = fmaf(2.0f, uF, m.ed) - e2;
    }
    const float beta = de * (1.0f / (2.0f * D));
    h[0] += (ddr - de) * LL::invw(0);
#pragma unroll
    for (int a = 0; a < D; ++a) {
        const int ip = LL::axis_plus(a);
        const float gam = 0.5f * ((m.j[a] + m.F[a]) - j2[a]);
        h[ip] += (beta + gam) * LL::invw(ip);
        h[ip + 1] += (beta - gam) * LL::invw(ip);
    }
}

// Eq. (4.4) collision, h* = (1 - om) h + om (f^eq / w_i - R_i(F)) + (1 - 1/(2 tau_hat)) S / w_i,
// with f^eq of Eq. (2.2) and S = F (Eq. 3.3) + H (Eq. 3.7) + P (Eq. 3.12),
// evaluated once per +/-c pair from its even and odd parts.
//   hc    = (1 - 1/Pr) rho theta / 2   (0 without the thermal source)
//   gT    = grad theta per lattice spacing
//   pc    = -(k / (2 D tau)) |F^SC|^2 / (c0^2 G psi^2)   (0 without it)
// CONSERVE = false skips the FP32 compensation: under 16-bit storage the
// rounding of the stored values is four orders of magnitude larger than the
// residual it removes, and unbiased.
template <class L, bool CONSERVE = true>
__device__ __forceinline__ void collide(const KParams& p, const Frame& fr, float (&h)[L::Q], const Macro& m,
                                        float hc, const float (&gT)[3], float pc)
{
    using LL = Lat<L>;
    constexpr int D = L::D;
    constexpr float Df = (float)D;
    const float ic = LL::ic0sq;
    const float uu = (m.u[0] * m.u[0] + m.u[1] * m.u[1] + m.u[2] * m.u[2]) * ic;
    const float UF = (m.u[0] * m.F[0] + m.u[1] * m.F[1] + m.u[2] * m.F[2]) * ic;
    const float thb = m.thb, dth = m.dth, thb0 = fr.thb;
    const float om = p.omega, ka = p.kappa, om1 = 1.0f - p.omega;
    const float orho = om * m.rho;
    const float odr = om * m.dr;
    const float U[3] = {m.u[0] * ic, m.u[1] * ic, m.u[2] * ic};
    const float Ph[3] = {m.F[0] * ic, m.F[1] * ic, m.F[2] * ic};

    // Per-shell coefficients of the even (dK0, K2) and odd (K1) parts of the
    // equilibrium bracket and of the force source (M1); HS, PS of H and P.
    // dK0 = K0 - (1 + t0) is the even bracket relative to the frame
    // (thb^2 - thb0^2 = dth (thb + thb0)); R0 = 1 + t0 of the frame.  The
    // velocities are ordered by shell, so each shell's coefficients are
    // formed just before its pairs and are dead after them (few registers
    // live at once).
    const float muu = -0.5f * uu;
    struct ShellCoef {
        float dK0, R0, K1, K2, M1, HS, PS;
    };
    auto shell_coef = [&](int s) {
        ShellCoef c;
        const float xx = (float)L::shell_c2[s] * ic;
        const float q2 = 0.125f * (xx * xx - 2.0f * (Df + 2.0f) * xx + Df * (Df + 2.0f));
        c.R0 = 1.0f + ref_t0<L>(xx, thb0);
        c.dK0 = muu + 0.125f * uu * uu + dth * (0.5f * (xx - Df) + q2 * (thb + thb0)) +
                thb * 0.25f * uu * ((Df + 2.0f) - xx);
        c.K1 = 1.0f + muu + 0.5f * thb * (xx - Df - 2.0f);
        c.K2 = 0.5f - 0.25f * uu + 0.25f * thb * (xx - Df - 4.0f);
        c.M1 = 1.0f + 0.5f * (thb * (xx - Df - 2.0f) - uu);
        c.HS = hc * (xx - Df - 2.0f);
        c.PS = pc * (xx - Df);
        return c;
    };
    // rest velocity
    {
        const ShellCoef c = shell_coef(0);
        h[0] = fmaf(om1, h[0], fmaf(orho, c.dK0, odr * c.R0) + ka * (c.PS - UF));
    }
#pragma unroll
    for (int s = 1; s < L::NS; ++s) {
        const ShellCoef c = shell_coef(s);
#pragma unroll
        for (int pp = 0; pp < L::NP; ++pp) {
            const int i = 1 + 2 * pp;
            if (L::shell[i] != s) continue;
            constexpr float sixth = 1.0f / 6.0f, c24 = 1.0f / 24.0f;
            float a = 0.f, b = 0.f, g = 0.f;
            if (L::cx[i]) { a = fmaf((float)L::cx[i], U[0], a); b = fmaf((float)L::cx[i], Ph[0], b); g = fmaf((float)L::cx[i], gT[0], g); }
            if (L::cy[i]) { a = fmaf((float)L::cy[i], U[1], a); b = fmaf((float)L::cy[i], Ph[1], b); g = fmaf((float)L::cy[i], gT[1], g); }
            if (L::cz[i]) { a = fmaf((float)L::cz[i], U[2], a); b = fmaf((float)L::cz[i], Ph[2], b); g = fmaf((float)L::cz[i], gT[2], g); }
            const float a2 = a * a;
            const float fe = fmaf(a2, fmaf(a2, c24, c.K2), c.dK0);
            const float fo = a * fmaf(a2, sixth, c.K1);
            const float se = fmaf(a, b, c.PS - UF);
            const float so = fmaf(b, fmaf(0.5f, a2, c.M1), fmaf(c.HS, g, -a * UF));
            const float E = fmaf(orho, fe, odr * c.R0) + ka * se;
            const float O = fmaf(orho, fo, ka * so);
            h[i] = fmaf(om1, h[i], E + O);
            h[i + 1] = fmaf(om1, h[i + 1], E - O);
        }
    }
    if (CONSERVE) conserve<L>(p, h, m);
}

// Pseudopotential of Eq. (3.8) in FP64: psi = sqrt(2 (p_EOS - rho c0^2) / (G c0^2)),
// with the van der Waals or the Carnahan-Starling (Eq. 5.9) pressure.
__device__ __forceinline__ double psi_eos(const KParams& p, double rho, double c0sq, bool& bad)
{
    double pe;
    if (p.eos == EOS_CS) {
        const double e = 0.25 * p.eos_b * rho;
        if (!(rho > 0.0) || !(e < 1.0)) { bad = true; return 0.0; }
        const double d = 1.0 - e;
        pe = rho * p.eos_T * (1.0 + e * (1.0 + e * (1.0 - e))) / (d * d * d) - p.eos_a * rho * rho;
    } else {
        const double br = p.eos_b * rho;
        if (!(rho > 0.0) || !(br < 1.0)) { bad = true; return 0.0; }
        pe = rho * p.eos_T / (1.0 - br) - p.eos_a * rho * rho;
    }
    const double arg = 2.0 * (pe - rho * c0sq) / (p.G * c0sq);
    if (!(arg >= 0.0)) { bad = true; return 0.0; }
    return sqrt(arg);
}

}  // namespace holb
