// Gradient-ascent follow-up of candidates: one Adam step on (ln Mc, f0, cos theta, phi, psi)
// per template, with per-template step sizes set from the statistic's resolution, and the
// best parameters seen so far kept beside the moving ones.
#include "tfsc_device.hpp"
#include "tfsc_kernels.hpp"

namespace tfsc {

// state[i][16] = m[5], v[5], best Upsilon, best (mc, f0, cos theta, phi, psi); a bank given in ln Mc is
// stepped in ln Mc directly (the best mc is kept as a chirp mass either way)
__global__ void k_follow_step(FollowLaunch a) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    double *s = a.state + 16 * i;
    double mc = a.ln_mc ? exp(a.ln_mc[i]) : a.mc[i], f0 = a.f0[i], ct = a.ct[i], ph = a.phi[i], ps = a.psi[i];
    const double up = a.stat[i];
    if (a.step == 1) {
        for (int p = 0; p < 10; ++p) s[p] = 0.0;
        s[10] = -INFINITY;
    }
    if (up > s[10]) {
        s[10] = up;
        s[11] = mc;
        s[12] = f0;
        s[13] = ct;
        s[14] = ph;
        s[15] = ps;
    }
    if (!(a.lr_scale > 0.0) || !params_valid(mc, a.eta[i], f0, ct, a.ci[i])) return;
    // resolution: delta f0 = 0.1 / T_seg, delta ln Mc = delta f0 / ((5/3) fdot0 T_obs),
    // 0.05 for the angles (cos theta in its own units)
    Track T;
    track_init(T, mc, a.eta[i], f0);
    double Phi, f, fd;
    track_at(T, 0.0, Phi, f, fd);
    const double Tobs = (double)a.Nt * a.dT;
    const double Tseg = Tobs / (double)a.nseg[i];
    const double df0 = 0.1 / Tseg;
    const double res[5] = {df0 / ((5.0 / 3.0) * fd * Tobs), df0, 0.05, 0.05, 0.05};
    const double b1 = 0.9, b2 = 0.999;
    const double c1 = 1.0 - pow(b1, (double)a.step), c2 = 1.0 - pow(b2, (double)a.step);
    double d[5];
    for (int p = 0; p < 5; ++p) {
        const double g = a.g_params[5 * i + p];
        if (!isfinite(g)) {
            d[p] = 0.0;
            continue;
        }
        s[p] = b1 * s[p] + (1.0 - b1) * g;
        s[5 + p] = b2 * s[5 + p] + (1.0 - b2) * g * g;
        const double mh = s[p] / c1, vh = s[5 + p] / c2;
        d[p] = vh > 0.0 ? a.lr_scale * res[p] * mh / sqrt(vh) : 0.0;  // ascent
    }
    const double lnmc = a.ln_mc ? a.ln_mc[i] + d[0] : 0.0;
    mc = a.ln_mc ? exp(lnmc) : mc * exp(d[0]);
    f0 = f0 + d[1];
    if (!(f0 > 0.0)) f0 = a.f0[i];
    ct = ct + d[2];
    ph = ph + d[3];
    ps = ps + d[4];
    // keep (cos theta, phi) on the sphere: reflect through a pole, turning phi by pi
    if (ct > 1.0) {
        ct = 2.0 - ct;
        ph += kPi;
    } else if (ct < -1.0) {
        ct = -2.0 - ct;
        ph += kPi;
    }
    ct = fmin(1.0, fmax(-1.0, ct));
    ph = ph - kTwoPi * floor(ph / kTwoPi);
    ps = ps - kPi * floor(ps / kPi);
    if (a.ln_mc)
        a.ln_mc[i] = lnmc;
    else
        a.mc[i] = mc;
    a.f0[i] = f0;
    a.ct[i] = ct;
    a.phi[i] = ph;
    a.psi[i] = ps;
}

hipError_t launch_follow_step(const FollowLaunch &L, hipStream_t st) {
    if (L.n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_follow_step, dim3((unsigned)((L.n + 255) / 256)), dim3(256), 0, st, L);
    return hipGetLastError();
}

}  // namespace tfsc
