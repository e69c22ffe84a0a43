// Host build of the device collision and its vector-Jacobian product, for
// CPU tests: the same source the kernels inline, compiled for the host.
// Test infrastructure only; the library does not use it.
#include "dmrt_device.hpp"
#include "dmrt_internal.hpp"

using namespace dmrt;

extern "C" {

// Post-collision populations of one node (FP64), coefficients from the
// library's parameter map.
int dmrt_host_collide(const dmrt_params* p, const dmrt_derived* d, const double* f, const double* g,
                      double* fs, double* gs)
{
    const Coef<double> c = make_coef<double>(*p, *d);
    double ff[9], gg[5], th, ux, uy;
    for (int i = 0; i < 9; ++i) ff[i] = f[i];
    for (int i = 0; i < 5; ++i) gg[i] = g[i];
    if (p->bc_mode == DMRT_BC_CAVITY) collide<double, false>(ff, gg, c, th, ux, uy);
    else collide<double, true>(ff, gg, c, th, ux, uy);
    for (int i = 0; i < 9; ++i) fs[i] = ff[i];
    for (int i = 0; i < 5; ++i) gs[i] = gg[i];
    return 0;
}

// lf, lg: adjoints of the post-collision populations in, of the
// pre-collision ones out (cavity coefficients).
int dmrt_host_collide_vjp(const dmrt_params* p, const dmrt_derived* d, const double* f, const double* g,
                          double* lf, double* lg)
{
    const Coef<double> c = make_coef<double>(*p, *d);
    double ff[9], gg[5], a[9], b[5];
    for (int i = 0; i < 9; ++i) { ff[i] = f[i]; a[i] = lf[i]; }
    for (int i = 0; i < 5; ++i) { gg[i] = g[i]; b[i] = lg[i]; }
    collide_vjp<double>(ff, gg, c, a, b);
    for (int i = 0; i < 9; ++i) lf[i] = a[i];
    for (int i = 0; i < 5; ++i) lg[i] = b[i];
    return 0;
}

}  // extern "C"
