// Host side of the kernel launchers: dispatch to the instantiation units,
// dominant-kernel bookkeeping, lattice tables and the 16-bit offset.
#include <hip/hip_runtime.h>
#include <stdio.h>

#include "holb_kernels.h"

namespace holb {

static hipError_t dispatch(const LaunchCtx& c, int op, const float* a = nullptr, const float* b = nullptr,
                           const float* d = nullptr, float* o1 = nullptr, float* o2 = nullptr,
                           float* o3 = nullptr, double* dout = nullptr)
{
    const bool sixteen = c.storage != ST_F32;
    if (c.lattice == 0)
        return sixteen ? dispatch_d2_16(c, op, a, b, d, o1, o2, o3, dout) : dispatch_d2_f32(c, op, a, b, d, o1, o2, o3, dout);
    if (c.lattice == 1)
        return sixteen ? dispatch_d3_16(c, op, a, b, d, o1, o2, o3, dout) : dispatch_d3_f32(c, op, a, b, d, o1, o2, o3, dout);
    return hipErrorInvalidValue;
}

hipError_t launch_init(const LaunchCtx& c, const float* rho, const float* u, const float* theta)
{
    return dispatch(c, 0, rho, u, theta);
}
hipError_t launch_step(const LaunchCtx& c) { return dispatch(c, 1); }
hipError_t launch_aux(const LaunchCtx& c) { return dispatch(c, 2); }
hipError_t launch_fields(const LaunchCtx& c, float* rho, float* u, float* theta)
{
    return dispatch(c, 3, nullptr, nullptr, nullptr, rho, u, theta);
}
hipError_t launch_reduce(const LaunchCtx& c, double* out_dev)
{
    return dispatch(c, 4, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, out_dev);
}
int reduce_blocks(const LaunchCtx& c) { return nblocks_for(c.kp.N); }

// The dominant kernel of a step is the collision of the cells away from the
// wall layers (every cell in a periodic domain).
void dominant_kernel(const LaunchCtx& c, char* name, size_t len, long long* cells)
{
    const int n = c.lattice == 1 ? c.kp.nz : c.kp.ny;
    const int planes = c.kp.walls ? n - 6 : n;
    if (cells) *cells = (long long)planes * c.kp.nlayer;
    // kernel template arguments as a profiler lists them
    if (name && len)
        snprintf(name, len, "k_step<%s,%d,%d,false,%d>", c.lattice == 1 ? "D3Q39" : "D2Q37", c.storage, c.family,
                 c.frames);
}

int num_variants(const LaunchCtx&) { return 6; }

bool variant_supported(const LaunchCtx&, int variant) { return variant >= 0 && variant <= 5; }

// ------------------------------------------------------- host-side tables

template <class L>
static void table_of(int* c, double* w, double* c0sq)
{
    for (int i = 0; i < L::Q; ++i) {
        if (c) {
            c[3 * i + 0] = L::cx[i];
            c[3 * i + 1] = L::cy[i];
            c[3 * i + 2] = L::cz[i];
        }
        if (w) w[i] = L::shell_w[L::shell[i]];
    }
    if (c0sq) *c0sq = L::c0sq;
}

int lattice_Q(int lattice) { return lattice == 0 ? D2Q37::Q : D3Q39::Q; }
int lattice_NS(int lattice) { return lattice == 0 ? D2Q37::NS : D3Q39::NS; }
int lattice_D(int lattice) { return lattice == 0 ? D2Q37::D : D3Q39::D; }
void lattice_table(int lattice, int* c, double* w, double* c0sq)
{
    if (lattice == 0) table_of<D2Q37>(c, w, c0sq);
    else table_of<D3Q39>(c, w, c0sq);
}

// Offset d_i = (f^eq_i(rho0, u0, theta0) - f^eq_i(rho0, 0, theta0)) / w_i of
// the 16-bit storage (Eq. 2.2 in FP64 on the host), in the library's velocity
// order: the stored values are then centred on the moving reference state.
template <class L>
static void dev_ref(double rho, const double* u, double theta, float* out)
{
    const double ic = 1.0 / L::c0sq, D = L::D;
    const double thb = theta - 1.0;
    auto t = [&](double a, double uu, double xx) {
        return a + 0.5 * a * a - 0.5 * uu + 0.5 * thb * (xx - D) + a * a * a / 6.0 - 0.5 * a * uu +
               0.5 * a * thb * (xx - (D + 2)) + a * a * a * a / 24.0 - 0.25 * a * a * uu + 0.125 * uu * uu +
               0.25 * thb * (a * a * (xx - (D + 4)) + uu * ((D + 2) - xx)) +
               0.125 * thb * thb * (xx * xx - 2.0 * (D + 2) * xx + D * (D + 2));
    };
    const double uu = (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]) * ic;
    for (int i = 0; i < L::Q; ++i) {
        const double a = (L::cx[i] * u[0] + L::cy[i] * u[1] + L::cz[i] * u[2]) * ic;
        const double xx = (L::cx[i] * L::cx[i] + L::cy[i] * L::cy[i] + L::cz[i] * L::cz[i]) * ic;
        out[i] = (float)(rho * (t(a, uu, xx) - t(0.0, 0.0, xx)));
    }
}

void deviation_reference(int lattice, double rho, const double* u, double theta, float* ref_out)
{
    if (lattice == 0) dev_ref<D2Q37>(rho, u, theta, ref_out);
    else dev_ref<D3Q39>(rho, u, theta, ref_out);
}

}  // namespace holb
