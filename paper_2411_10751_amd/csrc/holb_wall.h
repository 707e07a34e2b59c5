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

// Eq. (2.2) in FP64 for one state (u, theta - 1): the bracket 1 + t_i of any
// direction i, split into its even and odd parts per shell as in the
// collision, t_i = K0_s + a (1 + K1_s) + a^2 (1/2 + K2_s) + a^3 / 6 + a^4 / 24
// with a = c_i . u / c0^2 (Horner form with explicit fma).
template <class L>
struct Feq64 {
    double u[3];
    double K0[L::NS], K1[L::NS], K2[L::NS];
    __device__ __forceinline__ Feq64(const double (&uu)[3], double thb)
    {
        constexpr double D = L::D;
        const double ic = 1.0 / L::c0sq;
        u[0] = uu[0] * ic;
        u[1] = uu[1] * ic;
        u[2] = uu[2] * ic;
        const double U2 = fma(uu[0], u[0], fma(uu[1], u[1], uu[2] * u[2]));
#pragma unroll
        for (int s = 0; s < L::NS; ++s) {
            const double xx = (double)L::shell_c2[s] * ic;
            const double q2 = 0.125 * (xx * xx - 2.0 * (D + 2.0) * xx + D * (D + 2.0));
            K0[s] = fma(-0.5, U2, fma(0.125 * U2, U2, thb * fma(thb, q2, fma(0.25 * U2, (D + 2.0) - xx, 0.5 * (xx - D)))));
            K1[s] = fma(-0.5, U2, 0.5 * thb * (xx - (D + 2.0)));
            K2[s] = fma(-0.25, U2, 0.25 * thb * (xx - (D + 4.0)));
        }
    }
    __device__ __forceinline__ double bracket(int i) const
    {
        double a = 0.0;
        if (L::cx[i]) a = fma((double)L::cx[i], u[0], a);
        if (L::cy[i]) a = fma((double)L::cy[i], u[1], a);
        if (L::cz[i]) a = fma((double)L::cz[i], u[2], a);
        const int s = L::shell[i];
        const double p3 = fma(a, 1.0 / 24.0, 1.0 / 6.0);
        const double p2 = fma(a, p3, 0.5 + K2[s]);
        const double p1 = fma(a, p2, 1.0 + K1[s]);
        return fma(a, p1, 1.0 + K0[s]);
    }
};

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
    const double ir = 1.0 / rho;
    double uF = 0.0, uu = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double F = (body && a < L::D) ? rho * (double)p.g[a] : 0.0;
        m.u[a] = fma(0.5, F, j[a]) * ir;
        uF = fma(m.u[a], F, uF);
        uu = fma(m.u[a], m.u[a], uu);
    }
    m.theta = (p.flags & KF_ISO) ? 1.0 : fma(-rho, uu, e + uF) * ir * (1.0 / (L::D * L::c0sq));
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
    const Feq64<L> ft(tu, (p.flags & KF_ISO) ? 0.0 : T.theta - 1.0);
    // target equilibrium in the unknown slots (per w_i) and the local state
    double et[Q];
    double rl = K.rho, jl[3] = {K.j[0], K.j[1], K.j[2]}, el = K.e;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        if (!wall_unknown<L, SIDE>(i)) continue;
        et[i] = T.rho * ft.bracket(i);
        const double f = L::shell_w[L::shell[i]] * et[i];
        rl += f;
        if (L::cx[i]) jl[0] += (double)L::cx[i] * f;
        if (L::cy[i]) jl[1] += (double)L::cy[i] * f;
        if (L::cz[i]) jl[2] += (double)L::cz[i] * f;
        el += (double)Lat<L>::c2(i) * f;
    }
    const WallState loc = macro64<L>(p, rl, jl, el);
    const double lu[3] = {loc.u[0], loc.u[1], loc.u[2]};
    const Feq64<L> fl(lu, (p.flags & KF_ISO) ? 0.0 : loc.theta - 1.0);
    double m = 0.0, ja[3] = {K.j[0], K.j[1], K.j[2]}, ea = K.e;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        if (!wall_unknown<L, SIDE>(i)) continue;
        const int ib = Lat<L>::opp(i);
        // f_i / w_i - R_i(F) = h_ibar + f^eq_i(tgt) / w_i - f^eq_ibar(loc) / w_i (same shell, same R)
        const double hi = (double)h[ib] + (et[i] - loc.rho * fl.bracket(ib));
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

// Unknown at the node DIST (0, 1 or 2) layers from the wall of side SIDE: the
// populations whose source lies beyond the wall (DIST = 0: the wall node).
template <class L, int SIDE>
__host__ __device__ constexpr bool unknown_at(int dist, int i)
{
    return SIDE == 0 ? cnorm<L>(i) > dist : cnorm<L>(i) < -dist;
}

// Slots of the buffer of closed populations: the unknowns of the wall node,
// then those of the first and the second fluid boundary node, each in
// velocity order (slot[dist][i], -1 where i is known).
template <class L, int SIDE>
struct ClosedMap {
    int slot[3][L::Q];
    int count;
    constexpr ClosedMap() : slot{}, count(0)
    {
        for (int dd = 0; dd < 3; ++dd)
            for (int k = 0; k < L::Q; ++k) slot[dd][k] = unknown_at<L, SIDE>(dd, k) ? count++ : -1;
    }
};
template <class L, int SIDE>
inline constexpr ClosedMap<L, SIDE> closed_map{};

// Store / load the closed unknown populations of a node dist layers from the
// wall of side SIDE (cil: the node's cell within its layer).
template <class L, int SIDE>
__device__ __forceinline__ void store_closed(const KParams& p, int dist, int cil, const float (&h)[L::Q])
{
    static_assert(closed_map<L, SIDE>.count <= WCLOSED_SLOTS, "closed-population buffer too small");
    float* b = p.wclosed + (long long)SIDE * WCLOSED_SLOTS * p.nlayer + cil;
#pragma unroll
    for (int dd = 0; dd < 3; ++dd) {
        if (dd != dist) continue;
#pragma unroll
        for (int i = 0; i < L::Q; ++i) {
            const int s = closed_map<L, SIDE>.slot[dd][i];
            if (s >= 0) b[(long long)s * p.nlayer] = h[i];
        }
    }
}

template <class L, int SIDE>
__device__ __forceinline__ void load_closed(const KParams& p, int dist, int cil, float (&h)[L::Q])
{
    const float* b = p.wclosed + (long long)SIDE * WCLOSED_SLOTS * p.nlayer + cil;
#pragma unroll
    for (int dd = 0; dd < 3; ++dd) {
        if (dd != dist) continue;
#pragma unroll
        for (int i = 0; i < L::Q; ++i) {
            const int s = closed_map<L, SIDE>.slot[dd][i];
            if (s >= 0) h[i] = b[(long long)s * p.nlayer];
        }
    }
}

// Unknown at the fluid boundary node DIST (1 or 2) layers from the wall of
// side SIDE: the populations whose source lies beyond the wall.
template <class L, int SIDE, int DIST>
__host__ __device__ constexpr bool fluid_unknown(int i)
{
    return SIDE == 0 ? cnorm<L>(i) > DIST : cnorm<L>(i) < -DIST;
}

// Section 4.3, Eqs. (4.7)-(4.8), at a fluid boundary node DIST layers from
// the wall of side SIDE: the unknown populations become f_i = f_ibar +
// f^eq_i(tgt) - f^eq_ibar(loc), with tgt the node's own previous-step (rho,
// u[D], theta) and loc the state of the known populations plus the target
// equilibrium in the unknown slots.  FP64 throughout, like the wall node: the
// local state differs from the target by the small non-equilibrium part,
// which FP32 sums of the populations would blur.  Returns the rebuilt mass
// (absolute); after: the node's state after the closure.
template <class L, int SIDE, int DIST>
__device__ __forceinline__ double fluid_close_at(const KParams& p, const Frame& fr, float (&h)[L::Q],
                                                 const double* tgt, WallState& after)
{
    constexpr int Q = L::Q, D = L::D;
    const double fr_rho = fr.rho, fr_thb = fr.thb;
    double tu[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int a = 0; a < D; ++a) tu[a] = tgt[1 + a];
    const double trho = tgt[0];
    const Feq64<L> ft(tu, (p.flags & KF_ISO) ? 0.0 : tgt[1 + D] - 1.0);
    // sums over the known populations, then the local state with the target
    // equilibrium in the unknown slots
    double rk = 0.0, jk[3] = {0.0, 0.0, 0.0}, ek = 0.0;
    double rl = 0.0, jl[3] = {0.0, 0.0, 0.0}, el = 0.0;
    double et[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const double w = L::shell_w[L::shell[i]];
        if (fluid_unknown<L, SIDE, DIST>(i)) {
            et[i] = trho * ft.bracket(i);
            const double f = w * et[i];
            rl += f;
            if (L::cx[i]) jl[0] += (double)L::cx[i] * f;
            if (L::cy[i]) jl[1] += (double)L::cy[i] * f;
            if (L::cz[i]) jl[2] += (double)L::cz[i] * f;
            el += (double)Lat<L>::c2(i) * f;
        } else {
            const double f = w * ((double)h[i] + fr_rho * rest_bracket64<L>(L::shell[i], fr_thb));
            rk += f;
            if (L::cx[i]) jk[0] += (double)L::cx[i] * f;
            if (L::cy[i]) jk[1] += (double)L::cy[i] * f;
            if (L::cz[i]) jk[2] += (double)L::cz[i] * f;
            ek += (double)Lat<L>::c2(i) * f;
        }
    }
    rl += rk;
    el += ek;
#pragma unroll
    for (int a = 0; a < 3; ++a) jl[a] += jk[a];
    const WallState loc = macro64<L>(p, rl, jl, el);
    const double lu[3] = {loc.u[0], loc.u[1], loc.u[2]};
    const Feq64<L> fl(lu, (p.flags & KF_ISO) ? 0.0 : loc.theta - 1.0);
    double m = 0.0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        if (!fluid_unknown<L, SIDE, DIST>(i)) continue;
        const int ib = Lat<L>::opp(i);
        const double hi = (double)h[ib] + (et[i] - loc.rho * fl.bracket(ib));
        h[i] = (float)hi;
        const double f = L::shell_w[L::shell[i]] * (hi + fr_rho * rest_bracket64<L>(L::shell[i], fr_thb));
        m += f;
        if (L::cx[i]) jk[0] += (double)L::cx[i] * f;
        if (L::cy[i]) jk[1] += (double)L::cy[i] * f;
        if (L::cz[i]) jk[2] += (double)L::cz[i] * f;
        ek += (double)Lat<L>::c2(i) * f;
    }
    after = macro64<L>(p, rk + m, jk, ek);
    return m;
}

// The same for a node kw layers into a domain of nw layers along the wall
// normal (kw = 1, 2, nw - 3 or nw - 2); the layer is wave-uniform in the
// kernels that call this, so the branch costs nothing.
template <class L>
__device__ __forceinline__ double fluid_close(const KParams& p, const Frame& fr, float (&h)[L::Q], const double* tgt,
                                              int kw, int nw, WallState& after)
{
    if (kw == 1) return fluid_close_at<L, 0, 1>(p, fr, h, tgt, after);
    if (kw == 2) return fluid_close_at<L, 0, 2>(p, fr, h, tgt, after);
    if (kw == nw - 2) return fluid_close_at<L, 1, 1>(p, fr, h, tgt, after);
    return fluid_close_at<L, 1, 2>(p, fr, h, tgt, after);
}

// Temperature field of the gradient stencil (theta - theta0) from a node's
// FP64 state after the closure.
__device__ __forceinline__ float theta_field64(const KParams& p, const WallState& s)
{
    return (p.flags & KF_ISO) ? 0.0f : (float)((s.theta - 1.0) - (double)p.thb_ref);
}

// Chord iterations on one set of Jacobian factors before they are formed
// anew (a new Jacobian costs NV + 1 closures, a chord iteration one).
constexpr int CHORD_ITERS = 8;

// Wall-node target from the boundary conditions (see the header): unknowns
// v = (rho, the tangential components of u, theta; no theta when isothermal),
// NV of them; residuals (rebuilt mass - want, tangential u after closure -
// udes, theta after closure - thdes).  Newton's method (chord iterations)
// started from T, the previous step's solution, with the LU factors LU of the
// Jacobian the previous step used if have_lu (it changes little from step to
// step); when CHORD_ITERS chord iterations have not converged, or without
// factors, the Jacobian is formed anew by finite differences at the current
// point.
// The iteration stops when the update is below 1e-12 relative.  The Jacobian
// is diagonally dominant (about 0.3 on the diagonal, off-diagonal entries up
// to 0.19 between rho and theta), so the elimination needs no pivoting.
// Returns false if it does not converge within five rounds of factors; LU
// holds the factors used last.
template <class L, int SIDE, int NV>
__device__ __forceinline__ bool wall_solve(const KParams& p, const Frame& fr, float (&h)[L::Q], const WallKnown& K,
                                           double want, const double (&udes)[3], double thdes, WallState& T,
                                           double (&LU)[4][4], bool have_lu)
{
    constexpr int D = L::D, WN = D - 1;  // wall-normal axis
    // v[0] rho, v[1 .. D-1] tangential u (axes 0 .. D-2), v[D] theta
    auto state = [&](const double (&v)[NV]) {
        WallState S;
        S.rho = v[0];
        S.u[0] = S.u[1] = S.u[2] = 0.0;
#pragma unroll
        for (int a = 0; a < D - 1; ++a) S.u[a] = v[1 + a];
        S.u[WN] = udes[WN];
        S.theta = NV > D ? v[NV - 1] : 1.0;
        return S;
    };
    auto resid = [&](const double (&v)[NV], double (&r)[NV]) {
        WallState a;
        const double m = wall_close<L, SIDE, false>(p, fr, h, K, state(v), a);
        r[0] = m - want;
#pragma unroll
        for (int q = 1; q < D && q < NV; ++q) r[q] = a.u[q - 1] - udes[q - 1];
        if (NV > D) r[NV - 1] = a.theta - thdes;
    };
    double v[NV];
    v[0] = T.rho;
#pragma unroll
    for (int a = 0; a < D - 1; ++a) v[1 + a] = T.u[a];
    if (NV > D) v[NV - 1] = T.theta;
    double r[NV];
    resid(v, r);
    bool fresh = !have_lu;
    bool ok = false;
    for (int jac = 0; jac < 5 && !ok; ++jac) {
        if (fresh) {
#pragma unroll 1
            for (int c = 0; c < NV; ++c) {
                double vs[NV], rs[NV], hs = 0.0;
#pragma unroll
                for (int q = 0; q < NV; ++q) {
                    const bool on = q == c;
                    const double step = 1e-7 * (fabs(v[q]) + ((q > 0 && q < D) ? 1e-2 : 0.0));
                    hs = on ? step : hs;
                    vs[q] = on ? v[q] + step : v[q];
                }
                resid(vs, rs);
#pragma unroll
                for (int q = 0; q < NV; ++q) {
                    const double col = (rs[q] - r[q]) / hs;
#pragma unroll
                    for (int cc = 0; cc < NV; ++cc)
                        if (cc == c) LU[q][cc] = col;
                }
            }
            // LU factors in place (no pivoting)
#pragma unroll
            for (int k = 0; k < NV; ++k) {
                if (!(fabs(LU[k][k]) > 0.0)) return false;
#pragma unroll
                for (int q = k + 1; q < NV; ++q) {
                    LU[q][k] /= LU[k][k];
#pragma unroll
                    for (int c = k + 1; c < NV; ++c) LU[q][c] -= LU[q][k] * LU[k][c];
                }
            }
        }
        for (int it = 0; it < CHORD_ITERS; ++it) {
            double y[NV];
#pragma unroll
            for (int q = 0; q < NV; ++q) {
                double acc = -r[q];
#pragma unroll
                for (int c = 0; c < q; ++c) acc -= LU[q][c] * y[c];
                y[q] = acc;
            }
            bool done = true;
#pragma unroll
            for (int q = NV - 1; q >= 0; --q) {
                double acc = y[q];
#pragma unroll
                for (int c = q + 1; c < NV; ++c) acc -= LU[q][c] * y[c];
                y[q] = acc / LU[q][q];
                v[q] += y[q];
                if (!(fabs(y[q]) <= 1e-12 * (1.0 + fabs(v[q])))) done = false;
            }
            if (done) {
                ok = true;
                break;
            }
            resid(v, r);
        }
        fresh = true;
    }
    T = state(v);
    return ok;
}

}  // namespace holb
