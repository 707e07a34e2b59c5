// TMS wall closure (Section 4.3, Eqs. 4.7-4.8) in FP64, and the solve of the
// wall-node target from the boundary conditions.
//
// Walls are normal to the last axis.  The first layer next to each wall holds
// the wall nodes, outside the fluid; the wall lies half-way between them and
// the first fluid layer.  The unknown populations of a boundary node are
// rebuilt as f_i = f_ibar + f^eq_i(tgt) - f^eq_ibar(loc), with loc the state
// of the known populations plus the target equilibrium in the unknown slots
// (Eq. 4.8).  Fluid boundary nodes target their own previous-step state; a
// wall node's target is fixed by the boundary conditions of an impermeable,
// no-slip, isothermal wall at the half-way plane:
//   - the populations rebuilt along the column (wall node and both fluid
//     boundary nodes) carry the mass that left through the wall in the last
//     streaming (fixes rho_tgt);
//   - after the closure the wall node holds the reflection 2 u_wall - u_1
//     (components along the wall) and 2 theta_wall - theta_1 of the first
//     fluid node's previous-step fields (fixes the tangential u_tgt and
//     theta_tgt); the wall-normal u_tgt is that reflection itself.
// k_wall_fluid and k_wall_solve (holb_kernels.h) solve these conditions once
// per state; every pass then closes the wall node at the stored target, so
// that the passes agree bitwise.
#pragma once

#include "holb_device.h"

namespace holb {

// wall-normal component of velocity i
template <class L>
__host__ __device__ constexpr int cnorm(int i)
{
    return L::D == 3 ? L::cz[i] : L::cy[i];
}

// Unknown at the wall node of side 0 (low wall, first layer) or 1 (high wall,
// last layer): the populations streamed in from beyond the wall.
template <class L, int SIDE>
__host__ __device__ constexpr bool wall_unknown(int i)
{
    return SIDE == 0 ? cnorm<L>(i) > 0 : cnorm<L>(i) < 0;
}

// R_s(F) = 1 + t(u = 0, theta_F) of shell s in FP64 (the rest bracket of a
// frame; the absolute population is w_i (h_i + rho_F R_s)).
template <class L>
__device__ __forceinline__ double rest_bracket64(int s, double thb)
{
    constexpr double D = L::D;
    const double xx = (double)L::shell_c2[s] / L::c0sq;
    const double q2 = 0.125 * (xx * xx - 2.0 * (D + 2.0) * xx + D * (D + 2.0));
    return 1.0 + thb * (0.5 * (xx - D) + thb * q2);
}

// Sums over the known populations of a wall node (absolute, FP64): mass,
// momentum, energy moment sum |c|^2 f.
struct WallKnown {
    double rho, j[3], e;
};

// Target or after-closure state: rho, u[3], theta.
struct WallState {
    double rho, u[3], theta;
};

template <class L, int SIDE>
__device__ __forceinline__ WallKnown wall_known(const Frame& fr, const float (&h)[L::Q])
{
    WallKnown K{0.0, {0.0, 0.0, 0.0}, 0.0};
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        if (wall_unknown<L, SIDE>(i)) continue;
        const double w = L::shell_w[L::shell[i]];
        const double f = w * ((double)h[i] + (double)fr.rho * rest_bracket64<L>(L::shell[i], (double)fr.thb));
        K.rho += f;
        if (L::cx[i]) K.j[0] += (double)L::cx[i] * f;
        if (L::cy[i]) K.j[1] += (double)L::cy[i] * f;
        if (L::cz[i]) K.j[2] += (double)L::cz[i] * f;
        K.e += (double)Lat<L>::c2(i) * f;
    }
    return K;
}

// Macroscopic state of Eq. (4.5) from absolute moments (rho, j, e), with the
// body-force shift (F = rho g): rho u = j + F/2, rho D c0^2 theta = e - rho
// |u|^2 + u.F.
template <class L>
__device__ __forceinline__ WallState macro64(const KParams& p, double rho, const double (&j)[3], double e)
{
    WallState m;
    m.rho = rho;
    const bool body = p.flags & KF_BODY;
    double uF = 0.0, uu = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double F = (body && a < L::D) ? rho * (double)p.g[a] : 0.0;
        m.u[a] = (j[a] + 0.5 * F) / rho;
        uF += m.u[a] * F;
        uu += m.u[a] * m.u[a];
    }
    m.theta = (p.flags & KF_ISO) ? 1.0 : (e - rho * uu + uF) / (rho * (L::D * L::c0sq));
    return m;
}

// Closure of a wall node at target T (Eq. 4.7 with the local state of Eq.
// 4.8).  h: the node's pulled deviations in frame fr (unknown slots are not
// read); K: its known sums.  Writes the rebuilt deviations of the unknown
// slots to h if WRITE; returns the rebuilt mass and the state after closure.
template <class L, int SIDE, bool WRITE>
__device__ __forceinline__ double wall_close(const KParams& p, const Frame& fr, float (&h)[L::Q], const WallKnown& K,
                                             const WallState& T, WallState& after)
{
    constexpr int Q = L::Q;
    const double tu[3] = {T.u[0], T.u[1], T.u[2]};
    const double tthb = (p.flags & KF_ISO) ? 0.0 : T.theta - 1.0;
    // target equilibrium in the unknown slots (per w_i) and the local state
    double et[Q];
    double rl = K.rho, jl[3] = {K.j[0], K.j[1], K.j[2]}, el = K.e;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        if (!wall_unknown<L, SIDE>(i)) continue;
        et[i] = T.rho * (1.0 + feq_poly<L, double>(i, tu, tthb));
        const double f = L::shell_w[L::shell[i]] * et[i];
        rl += f;
        if (L::cx[i]) jl[0] += (double)L::cx[i] * f;
        if (L::cy[i]) jl[1] += (double)L::cy[i] * f;
        if (L::cz[i]) jl[2] += (double)L::cz[i] * f;
        el += (double)Lat<L>::c2(i) * f;
    }
    const WallState loc = macro64<L>(p, rl, jl, el);
    const double lu[3] = {loc.u[0], loc.u[1], loc.u[2]};
    const double lthb = (p.flags & KF_ISO) ? 0.0 : loc.theta - 1.0;
    double m = 0.0, ja[3] = {K.j[0], K.j[1], K.j[2]}, ea = K.e;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        if (!wall_unknown<L, SIDE>(i)) continue;
        const int ib = Lat<L>::opp(i);
        // f_i / w_i - R_i(F) = h_ibar + f^eq_i(tgt) / w_i - f^eq_ibar(loc) / w_i (same shell, same R)
        const double hi = (double)h[ib] + (et[i] - loc.rho * (1.0 + feq_poly<L, double>(ib, lu, lthb)));
        if (WRITE) h[i] = (float)hi;
        const double f = L::shell_w[L::shell[i]] * (hi + (double)fr.rho * rest_bracket64<L>(L::shell[i], (double)fr.thb));
        m += f;
        if (L::cx[i]) ja[0] += (double)L::cx[i] * f;
        if (L::cy[i]) ja[1] += (double)L::cy[i] * f;
        if (L::cz[i]) ja[2] += (double)L::cz[i] * f;
        ea += (double)Lat<L>::c2(i) * f;
    }
    after = macro64<L>(p, K.rho + m, ja, ea);
    return m;
}

// Section 4.3, Eqs. (4.7)-(4.8), at a fluid boundary node (second or third
// layer from a wall): the unknown populations (bit i of unk) become f_i =
// f_ibar + f^eq_i(tgt) - f^eq_ibar(loc), with tgt the node's own previous-step
// (rho, u[D], theta) and loc the state of the known populations plus the
// target equilibrium in the unknown slots.  FP64 throughout, like the wall
// node: the local state differs from the target by the small non-equilibrium
// part, which FP32 sums of the populations would blur.  Returns the rebuilt
// mass (absolute).
template <class L>
__device__ __forceinline__ double fluid_close(const KParams& p, const Frame& fr, float (&h)[L::Q], uint64_t unk,
                                              const double* tgt)
{
    constexpr int Q = L::Q, D = L::D;
    const double fr_rho = fr.rho, fr_thb = fr.thb;
    double tu[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int a = 0; a < D; ++a) tu[a] = tgt[1 + a];
    const double trho = tgt[0];
    const double tthb = (p.flags & KF_ISO) ? 0.0 : (double)tgt[1 + D] - 1.0;
    double rl = 0.0, jl[3] = {0.0, 0.0, 0.0}, el = 0.0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const double w = L::shell_w[L::shell[i]];
        const double f = ((unk >> i) & 1ull) ? w * trho * (1.0 + feq_poly<L, double>(i, tu, tthb))
                                             : w * ((double)h[i] + fr_rho * rest_bracket64<L>(L::shell[i], fr_thb));
        rl += f;
        if (L::cx[i]) jl[0] += (double)L::cx[i] * f;
        if (L::cy[i]) jl[1] += (double)L::cy[i] * f;
        if (L::cz[i]) jl[2] += (double)L::cz[i] * f;
        el += (double)Lat<L>::c2(i) * f;
    }
    const WallState loc = macro64<L>(p, rl, jl, el);
    const double lu[3] = {loc.u[0], loc.u[1], loc.u[2]};
    const double lthb = (p.flags & KF_ISO) ? 0.0 : loc.theta - 1.0;
    double m = 0.0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        if (!((unk >> i) & 1ull)) continue;
        const int ib = Lat<L>::opp(i);
        const double hi = (double)h[ib] + (trho * (1.0 + feq_poly<L, double>(i, tu, tthb)) -
                                           loc.rho * (1.0 + feq_poly<L, double>(ib, lu, lthb)));
        h[i] = (float)hi;
        m += L::shell_w[L::shell[i]] * (hi + fr_rho * rest_bracket64<L>(L::shell[i], fr_thb));
    }
    return m;
}

// Wall-node target from the boundary conditions (see the header): unknowns
// v = (rho, the tangential components of u, theta; no theta when isothermal),
// NV of them; residuals (rebuilt mass - want, tangential u after closure -
// udes, theta after closure - thdes).  Newton's method with a finite-
// difference Jacobian, started from T (the previous step's solution): the
// Jacobian is formed at the start and again after every four chord
// iterations that have not converged, and the iteration stops when the
// update is below 1e-12 relative.  The Jacobian is diagonally dominant (about
// 0.3 on the diagonal, off-diagonal entries up to 0.19 between rho and
// theta), so the elimination needs no pivoting.  Returns false if it does not
// converge within four Jacobians.
template <class L, int SIDE, int NV>
__device__ __forceinline__ bool wall_solve(const KParams& p, const Frame& fr, float (&h)[L::Q], const WallKnown& K,
                                           double want, const double (&udes)[3], double thdes, WallState& T)
{
    constexpr int D = L::D, WN = D - 1;  // wall-normal axis
    // variable q -> component: 0 rho, 1 .. D-1 tangential u (axes 0 .. D-2), D theta
    auto get = [&](const WallState& S, int q) -> double {
        return q == 0 ? S.rho : (q < D ? S.u[q - 1] : S.theta);
    };
    auto set = [&](WallState& S, int q, double v) {
        if (q == 0) S.rho = v;
        else if (q < D) S.u[q - 1] = v;
        else S.theta = v;
    };
    auto resid = [&](const WallState& S, double (&r)[NV]) {
        WallState a;
        const double m = wall_close<L, SIDE, false>(p, fr, h, K, S, a);
        r[0] = m - want;
#pragma unroll
        for (int q = 1; q < D && q < NV; ++q) r[q] = a.u[q - 1] - udes[q - 1];
        if (NV > D) r[NV - 1] = a.theta - thdes;
    };
    T.u[WN] = udes[WN];
    if (NV == D) T.theta = 1.0;
    double r[NV], J[NV][NV];
    resid(T, r);
    for (int jac = 0; jac < 4; ++jac) {
#pragma unroll
        for (int c = 0; c < NV; ++c) {
            WallState S = T;
            const double v = get(T, c);
            const double hs = 1e-7 * (fabs(v) + ((c > 0 && c < D) ? 1e-2 : 0.0));
            set(S, c, v + hs);
            double rs[NV];
            resid(S, rs);
#pragma unroll
            for (int q = 0; q < NV; ++q) J[q][c] = (rs[q] - r[q]) / hs;
        }
        // LU factors in place (no pivoting)
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            if (!(fabs(J[k][k]) > 0.0)) return false;
#pragma unroll
            for (int q = k + 1; q < NV; ++q) {
                J[q][k] /= J[k][k];
#pragma unroll
                for (int c = k + 1; c < NV; ++c) J[q][c] -= J[q][k] * J[k][c];
            }
        }
        for (int it = 0; it < 4; ++it) {
            double y[NV];
#pragma unroll
            for (int q = 0; q < NV; ++q) {
                double acc = -r[q];
#pragma unroll
                for (int c = 0; c < q; ++c) acc -= J[q][c] * y[c];
                y[q] = acc;
            }
            bool done = true;
#pragma unroll
            for (int q = NV - 1; q >= 0; --q) {
                double acc = y[q];
#pragma unroll
                for (int c = q + 1; c < NV; ++c) acc -= J[q][c] * y[c];
                y[q] = acc / J[q][q];
                const double v = get(T, q) + y[q];
                set(T, q, v);
                if (!(fabs(y[q]) <= 1e-12 * (1.0 + fabs(v)))) done = false;
            }
            if (done) return true;
            resid(T, r);
        }
    }
    return false;
}

}  // namespace holb
