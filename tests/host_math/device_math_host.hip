// Host build of the device collision and its vector-Jacobian product, for
// CPU tests: the same source the kernels inline, compiled for the host.
// Test infrastructure only; the library does not use it.
#include "dmrt_device.hpp"
#include "dmrt_internal.hpp"

using namespace dmrt;

namespace {

// The two ways the adjoint can form the transposed Jacobian at a node:
// (a) collide_vjp at the pre-collision state (f, g); (b) collide_vjp_at at
// the u, v, theta that the forward collision returns for that state (what
// the recompute stores).  Both results out (14 values each).
template <typename real>
static void vjp_paths(const dmrt_params* p, const dmrt_derived* d, const real* f, const real* g,
                      const real* lam, real* out_a, real* out_b)
{
    const Coef<real> c = make_coef<real>(*p, *d);
    real ff[9], gg[5], a[9], b[5];
    for (int i = 0; i < 9; ++i) { ff[i] = f[i]; a[i] = lam[i]; }
    for (int i = 0; i < 5; ++i) { gg[i] = g[i]; b[i] = lam[9 + i]; }
    collide_vjp<real>(ff, gg, c, a, b);
    for (int i = 0; i < 9; ++i) out_a[i] = a[i];
    for (int i = 0; i < 5; ++i) out_a[9 + i] = b[i];
    real th, ux, uy;
    collide<real>(ff, gg, c, th, ux, uy);
    for (int i = 0; i < 9; ++i) a[i] = lam[i];
    for (int i = 0; i < 5; ++i) b[i] = lam[9 + i];
    collide_vjp_at<real>(ux, uy, th, c, a, b);
    for (int i = 0; i < 9; ++i) out_b[i] = a[i];
    for (int i = 0; i < 5; ++i) out_b[9 + i] = b[i];
}

}  // namespace

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

int dmrt_host_vjp_paths_f64(const dmrt_params* p, const dmrt_derived* d, const double* f, const double* g,
                            const double* lam, double* out_a, double* out_b)
{
    vjp_paths<double>(p, d, f, g, lam, out_a, out_b);
    return 0;
}

int dmrt_host_vjp_paths_f32(const dmrt_params* p, const dmrt_derived* d, const float* f, const float* g,
                            const float* lam, float* out_a, float* out_b)
{
    vjp_paths<float>(p, d, f, g, lam, out_a, out_b);
    return 0;
}

}  // extern "C"
