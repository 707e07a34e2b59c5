// Host-side helpers shared by the single-run and batched C ABI files:
// error reporting, configuration checks and kernel parameters.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>

#include "../../include/holb.h"
#include "holb_internal.h"

namespace holb {

static_assert(EOS_VDW == HOLB_EOS_VDW && EOS_CS == HOLB_EOS_CS, "equation-of-state codes");

extern thread_local std::string g_last_error;

inline holb_status fail(holb_status code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

inline holb_status hip_fail(hipError_t e, const char* what)
{
    return fail(HOLB_EHIP, "%s: %s", what, hipGetErrorString(e));
}

constexpr size_t ALIGN = 256;
inline size_t align_up(size_t v, size_t a = ALIGN) { return (v + a - 1) / a * a; }

inline int family_of(uint32_t sources)
{
    if (sources & HOLB_SRC_PTENSOR) return FAM_PTENSOR;
    if (sources & HOLB_SRC_THERMAL) return FAM_THERMAL;
    return FAM_LOCAL;
}

inline holb_status validate(const holb_config* c)
{
    if (!c) return fail(HOLB_EINVAL, "config is NULL");
    if (c->abi_version != HOLB_ABI_VERSION)
        return fail(HOLB_EINVAL, "abi_version %d != %d", c->abi_version, HOLB_ABI_VERSION);
    if (c->lattice != HOLB_D2Q37 && c->lattice != HOLB_D3Q39) return fail(HOLB_EINVAL, "unknown lattice %d", c->lattice);
    if (c->nx < 1 || c->ny < 1 || c->nz < 1) return fail(HOLB_EINVAL, "grid dims must be >= 1");
    // lane offsets within a population plane are 32-bit byte offsets
    if ((long long)c->nx * c->ny * c->nz > (1ll << 29))
        return fail(HOLB_ESIZE, "grid of %lld cells exceeds 2^29", (long long)c->nx * c->ny * c->nz);
    if (c->lattice == HOLB_D2Q37 && c->nz != 1) return fail(HOLB_EINVAL, "D2Q37 needs nz == 1");
    const double N = (double)c->nx * c->ny * c->nz;
    if (N > 2147483647.0 / 1.0 || N * 39.0 > 9.0e15) return fail(HOLB_EINVAL, "grid too large");
    if (!(c->tau_hat > 0.5) || !std::isfinite(c->tau_hat)) return fail(HOLB_EINVAL, "tau_hat must be > 0.5");
    const uint32_t known = HOLB_SRC_BODY | HOLB_SRC_THERMAL | HOLB_SRC_PTENSOR;
    if (c->sources & ~known) return fail(HOLB_EINVAL, "unknown source bits 0x%x", c->sources);
    if (c->isothermal != 0 && c->isothermal != 1) return fail(HOLB_EINVAL, "isothermal must be 0 or 1");
    if (c->walls != 0 && c->walls != 1) return fail(HOLB_EINVAL, "walls must be 0 or 1");
    if (c->frames < HOLB_FRAMES_AUTO || c->frames > HOLB_FRAMES_CELL_U)
        return fail(HOLB_EINVAL, "frames must be one of HOLB_FRAMES_*");
    if (c->frames == HOLB_FRAMES_CELL_U && c->storage == HOLB_STORE_F32)
        return fail(HOLB_EUNSUPPORTED, "per-cell frames with momentum are for 16-bit storage only");
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(c->g[a])) return fail(HOLB_EINVAL, "g must be finite");
    if (c->grad_lag != 0 && c->grad_lag != 1) return fail(HOLB_EINVAL, "grad_lag must be 0 or 1");
    if (c->grad_lag && !(c->sources & HOLB_SRC_THERMAL))
        return fail(HOLB_EINVAL, "grad_lag applies to the thermal source only");
    if (c->sources & HOLB_SRC_THERMAL) {
        if (c->isothermal) return fail(HOLB_EUNSUPPORTED, "thermal source needs isothermal = 0");
        if (!(c->prandtl > 0) || !std::isfinite(c->prandtl)) return fail(HOLB_EINVAL, "prandtl must be > 0");
    }
    if (c->sources & HOLB_SRC_PTENSOR) {
        if (!c->isothermal) return fail(HOLB_EUNSUPPORTED, "pressure-tensor source runs in the isothermal mode");
        if (c->walls) return fail(HOLB_EUNSUPPORTED, "pressure-tensor source with walls is not supported");
        if (c->eos != HOLB_EOS_VDW && c->eos != HOLB_EOS_CS) return fail(HOLB_EINVAL, "eos must be one of HOLB_EOS_*");
        if (!(c->eos_b > 0) || !(c->eos_T > 0) || !(c->eos_a >= 0) || !std::isfinite(c->eos_a) ||
            !std::isfinite(c->eos_b) || !std::isfinite(c->eos_T))
            return fail(HOLB_EINVAL, "equation-of-state parameters need a >= 0, b > 0, T > 0");
        if (!(c->sc_G != 0) || !std::isfinite(c->sc_G)) return fail(HOLB_EINVAL, "sc_G must be non-zero");
        if (!std::isfinite(c->ptensor_k)) return fail(HOLB_EINVAL, "ptensor_k must be finite");
    }
    if (c->storage < HOLB_STORE_F32 || c->storage > HOLB_STORE_BF16DEV)
        return fail(HOLB_EINVAL, "unknown storage %d", c->storage);
    if (!(c->rho0 >= 0) || !std::isfinite(c->rho0)) return fail(HOLB_EINVAL, "rho0 must be finite and >= 0");
    if (!(c->theta0 > 0) || !std::isfinite(c->theta0)) return fail(HOLB_EINVAL, "theta0 must be > 0");
    if (c->storage != HOLB_STORE_F32) {
        if (!(c->rho0 > 0) || !(c->theta0 > 0) || !std::isfinite(c->theta0))
            return fail(HOLB_EINVAL, "deviation storage needs rho0 > 0 and theta0 > 0");
        for (int a = 0; a < 3; ++a)
            if (!std::isfinite(c->u0[a])) return fail(HOLB_EINVAL, "u0 must be finite");
    }
    if (c->walls) {
        const int nw = c->lattice == HOLB_D2Q37 ? c->ny : c->nz;
        if (nw < 8) return fail(HOLB_EINVAL, "walls need at least 8 layers along the wall-normal axis");
        for (int w = 0; w < 2; ++w) {
            if (!(c->theta_wall[w] > 0) && !c->isothermal) return fail(HOLB_EINVAL, "wall temperatures must be > 0");
            for (int a = 0; a < 3; ++a)
                if (!std::isfinite(c->u_wall[w][a])) return fail(HOLB_EINVAL, "wall velocity must be finite");
        }
    }
    return HOLB_OK;
}

// Frame mode of a configuration.  HOLB_FRAMES_AUTO takes, for the storage
// that keeps each workload within its tolerance at its horizon:
//   - walled domains: per-plane frames for FP32 and FP16 (the walls impose the
//     mean profile along the wall-normal axis), per-cell frames for BF16,
//     whose 8 significand bits need the closer frame;
//   - periodic domains with the pressure-tensor source: per-cell frames for
//     every storage (liquid and vapour share planes);
//   - other periodic domains: per-plane frames for FP32 and FP16 (no frame
//     words: the FP16 body-force step is 20% faster, at the same error), except
//     FP16 with the thermal source, which needs the cell's momentum in its
//     frame over long horizons (u 1.8e-3 against 3.7e-3 after 20,000 steps of
//     the thermal workload); per-cell frames for BF16.
inline int frames_of(const holb_config* c)
{
    if (c->frames == HOLB_FRAMES_CELL) return FM_CELL;
    if (c->frames == HOLB_FRAMES_PLANE) return FM_PLANE;
    if (c->frames == HOLB_FRAMES_CELL_U) return FM_CELLU;
    if (c->walls) return c->storage == HOLB_STORE_BF16DEV ? FM_CELL : FM_PLANE;
    if (c->sources & HOLB_SRC_PTENSOR) return FM_CELL;
    if (c->storage == HOLB_STORE_F32) return FM_PLANE;
    if (c->storage == HOLB_STORE_F16DEV) return (c->sources & HOLB_SRC_THERMAL) ? FM_CELLU : FM_PLANE;
    return FM_CELL;
}

inline KParams params_of(const holb_config* c)
{
    KParams p;
    memset(&p, 0, sizeof p);
    const int D = lattice_D(c->lattice);
    p.nx = c->nx; p.ny = c->ny; p.nz = c->nz;
    p.walls = c->walls;
    p.N = c->nx * c->ny * c->nz;
    p.nlayer = D == 2 ? c->nx : c->nx * c->ny;
    p.div_nx = make_fastdiv((unsigned)c->nx);
    p.div_ny = make_fastdiv((unsigned)c->ny);
    p.div_layer = make_fastdiv((unsigned)p.nlayer);
    p.flags = ((c->sources & HOLB_SRC_BODY) ? KF_BODY : 0u) | (c->isothermal ? KF_ISO : 0u);
    p.omega = (float)(1.0 / c->tau_hat);
    p.kappa = (float)(1.0 - 1.0 / (2.0 * c->tau_hat));
    for (int a = 0; a < 3; ++a) p.g[a] = (float)c->g[a];
    p.hfac = (c->sources & HOLB_SRC_THERMAL) ? (float)(0.5 * (1.0 - 1.0 / c->prandtl)) : 0.0f;
    for (int w = 0; w < 2; ++w) {
        p.twall[w] = (float)c->theta_wall[w];
        for (int a = 0; a < 3; ++a) p.uwall[w][a] = (float)c->u_wall[w][a];
    }
    double c0sq;
    lattice_table(c->lattice, nullptr, nullptr, &c0sq);
    if (c->sources & HOLB_SRC_PTENSOR) {
        const double tau = c->tau_hat - 0.5;
        p.pfac = -(c->ptensor_k / (2.0 * D * tau)) / (c0sq * c->sc_G);
        p.eos_a = c->eos_a; p.eos_b = c->eos_b; p.eos_T = c->eos_T; p.G = c->sc_G;
        p.eos = c->eos;
    }
    p.rho_ref = (float)c->rho0;
    // the reference temperature only where theta evolves
    p.thb_ref = c->isothermal ? 0.0f : (float)(c->theta0 - 1.0);
    if (c->storage != HOLB_STORE_F32) {
        double u0[3] = {c->u0[0], c->u0[1], D == 3 ? c->u0[2] : 0.0};
        deviation_reference(c->lattice, c->rho0, u0, c->isothermal ? 1.0 : c->theta0, p.dref);
        for (int a = 0; a < 3; ++a) p.u0s[a] = (float)(u0[a] / c0sq);
    }
    return p;
}

}  // namespace holb
