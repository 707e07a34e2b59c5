// Plain-old-data kernel parameters shared by the host runtime and the kernels.
#pragma once

#include <stdint.h>

namespace holb {

enum Storage { ST_F32 = 0, ST_F16 = 1, ST_BF16 = 2 };

// Source families select the kernel template (register footprint differs);
// the body force and the isothermal mode are runtime flags.
enum Family { FAM_LOCAL = 0, FAM_THERMAL = 1, FAM_PTENSOR = 2 };

enum : unsigned { KF_BODY = 1u, KF_ISO = 2u };

// How stored populations are referenced (see the frame section of
// holb_device.h): a frame per cell, kept beside the populations, the same
// with the cell's momentum added (16-bit storage), or a fixed frame per plane
// along the last axis, kept in a small table.
enum FrameMode { FM_CELL = 0, FM_PLANE = 1, FM_CELLU = 2 };

enum : unsigned { HOLB_ERR_DENSITY_BIT = 1u, HOLB_ERR_THETA_BIT = 2u, HOLB_ERR_EOS_BIT = 4u, HOLB_ERR_WALL_BIT = 8u };
// equation of state of the pseudopotential (values of HOLB_EOS_*)
enum : int { EOS_VDW = 0, EOS_CS = 1 };

constexpr int QMAX = 39;

// Division by a runtime constant d >= 1 for dividends n < 2^31, as a
// multiply-high, an add and a shift: with l = ceil(log2 d) and
// m = floor(2^32 (2^l - d) / d) + 1, n / d = (mulhi(n, m) + n) >> l
// (the round-up method of Granlund and Montgomery, 1994).
struct FastDiv {
    unsigned m, l, d;
};

inline FastDiv make_fastdiv(unsigned d)
{
    FastDiv f;
    f.d = d;
    f.l = 0;
    while ((1ull << f.l) < d) ++f.l;
    f.m = (unsigned)(((1ull << 32) * ((1ull << f.l) - d)) / d + 1);
    return f;
}

__host__ __device__ inline unsigned fastdiv(unsigned n, const FastDiv& f)
{
    const unsigned t = (unsigned)(((unsigned long long)n * f.m) >> 32);
    return (t + n) >> f.l;
}

struct KParams {
    int nx, ny, nz;      // grid
    int walls;           // 1: TMS walls normal to the last axis
    int N;               // cells
    int nlayer;          // cells per wall-normal layer (nx for 2D, nx*ny for 3D)
    FastDiv div_nx, div_ny, div_layer;
    long long pitch;     // elements per population plane
    unsigned flags;      // KF_*
    float omega, kappa;  // 1/tau_hat and 1 - 1/(2 tau_hat)
    float g[3];          // body-force acceleration
    float hfac;          // (1 - 1/Pr) / 2
    float twall[2];
    float uwall[2][3];
    double pfac;         // -(k / (2 D tau)) / (c0^2 G), tau = tau_hat - 1/2
    double eos_a, eos_b, eos_T, G;
    int eos;             // EOS_VDW or EOS_CS
    float rho_ref;       // rho0 and theta0 - 1 of the reference state: populations
    float thb_ref;       //   are handled as h_i = f_i / w_i - f^eq_i(rho0, 0, theta0) / w_i
    float dref[QMAX];    // d_i = (f^eq_i(rho0, u0, theta0) - f^eq_i(rho0, 0, theta0)) / w_i (16-bit offset)
    float u0s[3];        // u0 / c0^2: FM_CELLU frames carry rho (u - u0) / c0^2
    unsigned* err;       // device error word
    // FM_PLANE: rho and theta - 1 of each plane along the last axis (2 floats
    // per plane), and the shifts R_s(frame(m - c_m)) - R_s(frame(m)) at
    // [(m * 7 + c_m + 3) * NS + s] for plane m, last-axis velocity component c_m, shell s
    const float* plane_frame;
    const float* plane_shift;
    // Walled domains: the wall-node targets solved for the current state
    // (FP64, [side][WSOL_COMPS][cell in layer]: rho, u[3], theta, then the LU
    // factors of the Jacobian used, 4 x 4 row-major), and the mass rebuilt by
    // the closure of the two fluid boundary layers of each wall
    // ([side][distance 1, 2 from the wall][cell in layer]).
    double* wsol;
    double* mflu;
    // The closed unknown populations of the three boundary layers of each
    // wall (deviations h, FP32, [side][closed_slot][cell in layer]), written
    // by the solve and read by every pass over the state.
    float* wclosed;
};

// Slots of the closed-population buffer per wall and column (at most: 18 for
// D3Q39, 15 + 7 + 3 for D2Q37).
constexpr int WCLOSED_SLOTS = 32;

// Wall targets: 8 slots x (D + 2) components x nlayer cells, doubles, laid out
// [slot][component][cell in layer].  Slots 0-5 hold the previous-step rho,
// u[D], theta of the 6 boundary layers (3 per wall, wall_slot); slots 6 and
// 7 the wall-node target solved in the previous step at the low and high
// wall (the starting point of the next solve).  Then, per wall, the LU factors
// of the Jacobian that solve used ([side][16][cell in layer]; all zero before
// the first solve).
constexpr int TGT_SLOTS = 8;
constexpr int WSOL_COMPS = 21;
__host__ __device__ inline long long tgt_lu_offset(int D, int side, int nlayer)
{
    return ((long long)TGT_SLOTS * (D + 2) + 16LL * side) * nlayer;
}
__host__ __device__ inline int wall_slot(int k, int n)
{
    return k < 3 ? k : (k >= n - 3 ? k - (n - 6) : -1);
}
__host__ __device__ inline int warm_slot(int side) { return 6 + side; }

}  // namespace holb
