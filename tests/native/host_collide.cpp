// Host build of the device collision, for CPU tests that compare it with the
// oracle before any GPU run.  Test code only.
#include "../../paper_0903_5067_amd/csrc/lbmd_device.hpp"
#include <cmath>

template <typename R>
static void fill_const(lbd::CollideConst<R>& cc, double rho0, double ws, double wb, double wg,
                       double kT, double tau, int therm)
{
    const double b[19] = {1, 1. / 3, 1. / 3, 1. / 3, 2. / 3, 4. / 3, 4. / 9, 1. / 9, 1. / 9, 1. / 9,
                          2. / 3, 2. / 3, 2. / 3, 2. / 9, 2. / 9, 2. / 9, 2, 4. / 3, 4. / 9};
    double gb = 1 - wb, gs = 1 - ws, gg = 1 - wg;
    cc.rho0 = (R)rho0; cc.gb = (R)gb; cc.gs = (R)gs; cc.gg = (R)gg;
    cc.hb = (R)(0.5 * (1 + gb)); cc.hs = (R)(0.5 * (1 + gs));
    cc.mu = (R)(3.0 * kT * tau * tau);
    cc.therm = therm;
    for (int k = 0; k < 19; k++) {
        double g = k == 4 ? gb : (k < 10 ? gs : gg);
        cc.q[k] = k < 4 ? (R)0 : (R)std::sqrt((1 - g * g) / b[k]);
    }
}

extern "C" void host_collide_f64(const double* n, const double* dp, double rho0, double ws, double wb,
                                 double wg, double kT, double tau, int therm, unsigned node,
                                 unsigned step, unsigned k0, unsigned k1, double* out)
{
    lbd::CollideConst<double> cc;
    fill_const(cc, rho0, ws, wb, wg, kT, tau, therm);
    double d[19], o[19];
    for (int i = 0; i < 19; i++) d[i] = n[i] - lbd::wv(i) * rho0;
    lbd::collide<double>(d, o, dp[0], dp[1], dp[2], cc, node, step, k0, k1);
    for (int i = 0; i < 19; i++) out[i] = o[i] + lbd::wv(i) * rho0;
}

extern "C" void host_collide_f32(const double* n, const double* dp, double rho0, double ws, double wb,
                                 double wg, double kT, double tau, int therm, unsigned node,
                                 unsigned step, unsigned k0, unsigned k1, double* out)
{
    lbd::CollideConst<float> cc;
    fill_const(cc, rho0, ws, wb, wg, kT, tau, therm);
    float d[19], o[19];
    for (int i = 0; i < 19; i++) d[i] = (float)(n[i] - lbd::wv(i) * rho0);
    lbd::collide<float>(d, o, (float)dp[0], (float)dp[1], (float)dp[2], cc, node, step, k0, k1);
    for (int i = 0; i < 19; i++) out[i] = (double)o[i] + lbd::wv(i) * rho0;
}
