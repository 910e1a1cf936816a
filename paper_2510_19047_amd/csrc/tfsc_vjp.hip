// Vector-Jacobian product of the statistic with respect to (ln Mc, f0, cos theta, phi, psi).
//
// For L = sum_n g_n Upsilon_n with Upsilon_n = 2 |z_n|^2 / N_n (Eq. (Upsilon-seg)),
//   dL = sum_n sum_{pixels of n} Re[(a_n conj(D) - b_n conj(Y)) dY],
//   a_n = 4 g_n conj(z_n) / N_n,  b_n = 4 g_n |z_n|^2 / N_n^2,
// with (z_n, N_n) taken from the forward pass.  Nothing per pixel is stored: each
// wave recomputes its template's track, tranche spectra and response with
// forward-mode tangents (FP64 dual numbers) and contracts them with the adjoint
// on the fly, one lane per tranche as in the forward WAVE schedule.
//
// Per tranche, with H_k = h_k u_k w_m (channel independent) and Y_ck = T_c H_k:
//   G_c    = sum_k adj_ck H_k        = a S1_c - b conj(T_c) S2
//   J_c,p  = sum_k adj_ck dH_k/dp    = a U_c,p - b conj(T_c) V_p
//   dL/dp += Re(dT_c/dp G_c) + Re(T_c J_c,p),
// S1_c = sum conj(D_ck) H_k, S2 = sum |H_k|^2, U_c,p = sum conj(D_ck) dH_k/dp,
// V_p = sum conj(H_k) dH_k/dp.
//
// A phase shift common to all pixels of a segment leaves Upsilon_n unchanged, so
// the phase tangent of tranche m is taken relative to the segment's first tranche
// (dPhi_m - dPhi_ref).  This is exact in real arithmetic and removes the large
// common part of dPhi/d ln Mc (phase counted from coalescence) before it meets
// rounding in the adjoint.
#include "tfsc_device.hpp"
#include "tfsc_kernels.hpp"

// The tangent arithmetic below contracts multiply-adds into FMAs.  The FP64 track that fixes
// the integer structure (track_step, from tfsc_device.hpp, included above) is not affected.
#pragma clang fp contract(fast)

namespace tfsc {

// ------------------------------------------------------------------ dual numbers
template <int N>
struct Dn {
    double v;
    double d[N];
};

template <int N>
__device__ __forceinline__ Dn<N> dconst(double v) {
    Dn<N> r;
    r.v = v;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = 0.0;
    return r;
}
template <int N>
__device__ __forceinline__ Dn<N> operator+(Dn<N> a, Dn<N> b) {
    Dn<N> r;
    r.v = a.v + b.v;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = a.d[i] + b.d[i];
    return r;
}
template <int N>
__device__ __forceinline__ Dn<N> operator-(Dn<N> a, Dn<N> b) {
    Dn<N> r;
    r.v = a.v - b.v;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = a.d[i] - b.d[i];
    return r;
}
template <int N>
__device__ __forceinline__ Dn<N> operator-(Dn<N> a) {
    Dn<N> r;
    r.v = -a.v;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = -a.d[i];
    return r;
}
template <int N>
__device__ __forceinline__ Dn<N> operator*(Dn<N> a, Dn<N> b) {
    Dn<N> r;
    r.v = a.v * b.v;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i];
    return r;
}
template <int N>
__device__ __forceinline__ Dn<N> operator*(Dn<N> a, double s) {
    Dn<N> r;
    r.v = a.v * s;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * s;
    return r;
}
template <int N>
__device__ __forceinline__ Dn<N> operator*(double s, Dn<N> a) {
    return a * s;
}
template <int N>
__device__ __forceinline__ Dn<N> operator+(Dn<N> a, double s) {
    a.v += s;
    return a;
}
template <int N>
__device__ __forceinline__ Dn<N> operator+(double s, Dn<N> a) {
    a.v += s;
    return a;
}
template <int N>
__device__ __forceinline__ Dn<N> operator-(double s, Dn<N> a) {
    return (-a) + s;
}
template <int N>
__device__ __forceinline__ Dn<N> drcp(Dn<N> a) {
    const double r = 1.0 / a.v, r2 = -r * r;
    Dn<N> o;
    o.v = r;
#pragma unroll
    for (int i = 0; i < N; ++i) o.d[i] = a.d[i] * r2;
    return o;
}
template <int N>
__device__ __forceinline__ Dn<N> dsqrt(Dn<N> a) {
    const double s = sqrt(a.v), h = 0.5 / s;
    Dn<N> o;
    o.v = s;
#pragma unroll
    for (int i = 0; i < N; ++i) o.d[i] = a.d[i] * h;
    return o;
}
// reduce a revolution count to [-1/2, 1/2]; the tangent is unchanged
template <int N>
__device__ __forceinline__ Dn<N> dfrac(Dn<N> a) {
    a.v = frac_rev(a.v);
    return a;
}
// sin(2 pi r) for revolutions r
template <int N>
__device__ __forceinline__ Dn<N> dsin_rev(Dn<N> r) {
    double s, c;
    sincospi(2.0 * r.v, &s, &c);
    Dn<N> o;
    o.v = s;
#pragma unroll
    for (int i = 0; i < N; ++i) o.d[i] = kTwoPi * c * r.d[i];
    return o;
}
// sin(x)/x
template <int N>
__device__ __forceinline__ Dn<N> dsinc(Dn<N> x) {
    double v, dv;
    if (fabs(x.v) < 1e-4) {
        v = 1.0 - x.v * x.v * (1.0 / 6.0);
        dv = -x.v * (1.0 / 3.0);
    } else {
        double s, c;
        sincos(x.v, &s, &c);
        v = s / x.v;
        dv = (c - v) / x.v;
    }
    Dn<N> o;
    o.v = v;
#pragma unroll
    for (int i = 0; i < N; ++i) o.d[i] = dv * x.d[i];
    return o;
}

template <int N>
struct CDn {
    Dn<N> re, im;
};
template <int N>
__device__ __forceinline__ CDn<N> cdmul(CDn<N> a, CDn<N> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <int N>
__device__ __forceinline__ CDn<N> cdadd(CDn<N> a, CDn<N> b) {
    return {a.re + b.re, a.im + b.im};
}
template <int N>
__device__ __forceinline__ CDn<N> cdsub(CDn<N> a, CDn<N> b) {
    return {a.re - b.re, a.im - b.im};
}
template <int N>
__device__ __forceinline__ CDn<N> cdscale(CDn<N> a, Dn<N> s) {
    return {a.re * s, a.im * s};
}
template <int N>
__device__ __forceinline__ CDn<N> cdscale(CDn<N> a, double s) {
    return {a.re * s, a.im * s};
}
// e^{2 pi i r}
template <int N>
__device__ __forceinline__ CDn<N> dexpi_rev(Dn<N> r) {
    double s, c;
    sincospi(2.0 * r.v, &s, &c);
    CDn<N> o;
    o.re.v = c;
    o.im.v = s;
#pragma unroll
    for (int i = 0; i < N; ++i) {
        o.re.d[i] = -kTwoPi * s * r.d[i];
        o.im.d[i] = kTwoPi * c * r.d[i];
    }
    return o;
}

// ------------------------------------------------------------------ track tangents
// Tangent slots: 0 = ln Mc, 1 = f0 (eta is held fixed).  M scales with Mc, so
// dM/M = (1, 0); theta0 follows from theta0^3 P(theta0) = 8 pi M f0 by implicit
// differentiation; t_c = 5 M theta0^-8 / eta.
struct TrackTan {
    double mu[2];   // dM/M
    double dtc[2];  // dt_c
};

__device__ inline TrackTan track_tangents(const Track &T, double f0) {
    TrackTan G;
    const double th = T.th0, th2 = th * th, th3 = th2 * th, th4 = th2 * th2;
    const double dP = ((3.0 + (5.0 * T.a2) * th2) + (6.0 * T.a3) * th3) + (7.0 * T.a4) * th4;
    const double z = T.c8 * f0;
    const double dz[2] = {z, T.c8};
    G.mu[0] = 1.0;
    G.mu[1] = 0.0;
#pragma unroll
    for (int p = 0; p < 2; ++p) {
        const double dth0 = dz[p] / (th2 * dP);
        G.dtc[p] = T.tc * (G.mu[p] - 8.0 * dth0 / th);
    }
    return G;
}

// Phase, frequency, chirp and amplitude tangents at t < t_c (values come from track_at).
struct TrackDual {
    double dPhi[2], df[2], dfdot[2], dA[2];
};

__device__ inline TrackDual track_dual(const Track &T, const TrackTan &G, double t, double f) {
    const double tau = T.tc - t;
    const double q = (T.eta * tau) / (5.0 * T.M);
    const double th = 1.0 / sqrt(sqrt(sqrt(q)));
    const double th2 = th * th, th3 = th2 * th, th4 = th2 * th2, th5 = th4 * th, th9 = th5 * th4;
    const double dPf = ((3.0 + (5.0 * T.a2) * th2) + (6.0 * T.a3) * th3) + (7.0 * T.a4) * th4;
    const double ddPf = ((10.0 * T.a2) * th + (18.0 * T.a3) * th2) + (28.0 * T.a4) * th3;
    const double dfdth = (th2 / T.c8) * dPf;
    const double dthdt = (T.eta * th9) / (40.0 * T.M);
    const double Pp = ((1.0 + T.b2 * th2) + T.b3 * th3) + T.b4 * th4;
    const double dPp = ((2.0 * T.b2) * th + (3.0 * T.b3) * th2) + (4.0 * T.b4) * th3;
    const double dPhidth = (2.0 / T.eta) * (5.0 * Pp - th * dPp) / (th5 * th);
    const double A = pow(f, 2.0 / 3.0);
    TrackDual D;
#pragma unroll
    for (int p = 0; p < 2; ++p) {
        const double mu = G.mu[p];
        const double dth = -0.125 * th * (G.dtc[p] / tau - mu);
        D.df[p] = dfdth * dth - f * mu;
        const double d_dfdth = ((2.0 * th * dPf + th2 * ddPf) / T.c8) * dth - dfdth * mu;
        const double d_dthdt = dthdt * (9.0 * dth / th - mu);
        D.dfdot[p] = d_dfdth * dthdt + dfdth * d_dthdt;
        D.dPhi[p] = dPhidth * dth;
        D.dA[p] = (2.0 / 3.0) * (A / f) * D.df[p];
    }
    return D;
}

__device__ inline void dphi_at(const Track &T, const TrackTan &G, double t, double out[2]) {
    const double tau = T.tc - t;
    const double q = (T.eta * tau) / (5.0 * T.M);
    const double th = 1.0 / sqrt(sqrt(sqrt(q)));
    const double th2 = th * th, th3 = th2 * th, th4 = th2 * th2, th5 = th4 * th;
    const double Pp = ((1.0 + T.b2 * th2) + T.b3 * th3) + T.b4 * th4;
    const double dPp = ((2.0 * T.b2) * th + (3.0 * T.b3) * th2) + (4.0 * T.b4) * th3;
    const double dPhidth = (2.0 / T.eta) * (5.0 * Pp - th * dPp) / (th5 * th);
#pragma unroll
    for (int p = 0; p < 2; ++p) out[p] = dPhidth * (-0.125 * th * (G.dtc[p] / tau - G.mu[p]));
}

// ------------------------------------------------------------------ response tangents
// Tangent slots: 0 = f, 1 = cos theta, 2 = phi, 3 = psi.  Same formulas as transfer_ae.
struct SkyD {
    Dn<4> k[3], u[3], v[3], c2, s2;
    double ap, ci;
};

__device__ inline void sky_dual(SkyD &S, double ct, double phi, double psi, double ci) {
    Dn<4> c = dconst<4>(ct);
    c.d[1] = 1.0;
    double sp, cp, s2, c2;
    sincos(phi, &sp, &cp);
    sincos(2.0 * psi, &s2, &c2);
    Dn<4> Sp = dconst<4>(sp), Cp = dconst<4>(cp);
    Sp.d[2] = cp;
    Cp.d[2] = -sp;
    Dn<4> st = dsqrt(1.0 - c * c);
    S.k[0] = -(st * Cp);
    S.k[1] = -(st * Sp);
    S.k[2] = -c;
    S.u[0] = c * Cp;
    S.u[1] = c * Sp;
    S.u[2] = -st;
    S.v[0] = Sp;
    S.v[1] = -Cp;
    S.v[2] = dconst<4>(0.0);
    S.c2 = dconst<4>(c2);
    S.s2 = dconst<4>(s2);
    S.c2.d[3] = -2.0 * s2;
    S.s2.d[3] = 2.0 * c2;
    S.ap = (1.0 + ci * ci) / 2.0;
    S.ci = ci;
}

template <bool WITH_T>
__device__ inline void transfer_ae_dual(const SkyD &S, const double (&g)[kGeoRows], double f, CDn<4> &TA,
                                        CDn<4> &TE, CDn<4> &TT) {
    const double L = kArmM / kClight;
    Dn<4> F = dconst<4>(f);
    F.d[0] = 1.0;
    Dn<4> kp[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        kp[i] = S.k[0] * g[3 * i] + S.k[1] * g[3 * i + 1] + S.k[2] * g[3 * i + 2];
    }
    const Dn<4> pfL = F * (kPi * L);
    CDn<4> Gd[3], Gr[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int s = a, r = (a + 1) % 3;
        const double n0 = g[9 + 3 * a + 0];
        const double n1 = g[9 + 3 * a + 1];
        const double n2 = g[9 + 3 * a + 2];
        Dn<4> kn = S.k[0] * n0 + S.k[1] * n1 + S.k[2] * n2;
        Dn<4> nu = S.u[0] * n0 + S.u[1] * n1 + S.u[2] * n2;
        Dn<4> nv = S.v[0] * n0 + S.v[1] * n1 + S.v[2] * n2;
        Dn<4> xp0 = nu * nu - nv * nv, xx0 = 2.0 * (nu * nv);
        Dn<4> xp = S.c2 * xp0 + S.s2 * xx0;
        Dn<4> xx = S.s2 * (-xp0) + S.c2 * xx0;
        CDn<4> amp = {xp * S.ap, xx * (-S.ci)};
        Dn<4> rev = dfrac(F * (-0.5) * ((kp[s] + kp[r]) + L));
        CDn<4> Ea = cdmul(dexpi_rev(rev), amp);
        CDn<4> B = {pfL * Ea.im, -(pfL * Ea.re)};
        Gd[a] = cdscale(B, dsinc(pfL * (1.0 - kn)));
        Gr[a] = cdscale(B, dsinc(pfL * (1.0 + kn)));
    }
    const CDn<4> G01 = Gd[0], G10 = Gr[0], G12 = Gd[1], G21 = Gr[1], G20 = Gd[2], G02 = Gr[2];
    // 1 - D^2 = 2 i sin(2 pi f L) D, D = e^{-2 pi i f L}
    const Dn<4> rl = dfrac(F * L);
    const CDn<4> D = dexpi_rev(-rl);
    const Dn<4> s2 = dsin_rev(rl);
    const CDn<4> om = {(-2.0) * (s2 * D.im), 2.0 * (s2 * D.re)};
    const CDn<4> TX = cdmul(om, cdsub(cdadd(G20, cdmul(D, G02)), cdadd(G10, cdmul(D, G01))));
    const CDn<4> TY = cdmul(om, cdsub(cdadd(G01, cdmul(D, G10)), cdadd(G21, cdmul(D, G12))));
    const CDn<4> TZ = cdmul(om, cdsub(cdadd(G12, cdmul(D, G21)), cdadd(G02, cdmul(D, G20))));
    const double is2 = 0.70710678118654752440, is6 = 0.40824829046386301637;
    TA = cdscale(cdsub(TZ, TX), is2);
    TE = cdscale(cdadd(cdsub(TX, cdscale(TY, 2.0)), TZ), is6);
    if constexpr (WITH_T) TT = cdscale(cdadd(cdadd(TX, TY), TZ), 0.57735026918962576451);  // (X + Y + Z) / sqrt3
}

// ------------------------------------------------------------------ spectrum tangents
// Tangent slots: 0 = ln Mc, 1 = f0.  Bin-relative Fresnel form as in tranche_spectrum_bin.
struct SpecD {
    Dn<2> x, beta, s, P, Q, hib;
    CDn<2> E0, E1;
    double rev0, drev0[2];
    double r6;
};

__device__ inline int spec_dual(SpecD &S, double Phi, double f, double fdot, const TrackDual &D, const double dref[2],
                                double dT) {
    const double fT = f * dT;
    const double kc = ceil(fT);
    S.x = dconst<2>(fT - kc);
    S.beta = dconst<2>((fdot * dT) * dT);
    Dn<2> A = dconst<2>(pow(f, 2.0 / 3.0)), Fd = dconst<2>(fdot);
    Dn<2> r0 = dconst<2>(phase_to_rev(Phi));
#pragma unroll
    for (int p = 0; p < 2; ++p) {
        S.x.d[p] = dT * D.df[p];
        S.beta.d[p] = (dT * dT) * D.dfdot[p];
        A.d[p] = D.dA[p];
        Fd.d[p] = D.dfdot[p];
        r0.d[p] = (D.dPhi[p] - dref[p]) * (1.0 / kTwoPi);
    }
    S.s = dsqrt(2.0 * drcp(S.beta));
    S.P = A * drcp(dsqrt(2.0 * Fd));
    S.Q = A * (dT / kTwoPi);
    S.hib = 0.5 * drcp(S.beta);
    S.r6 = 6.0 / S.s.v;
    Dn<2> r1 = dfrac(r0 + S.x + 0.5 * S.beta);
    S.E0 = dexpi_rev(r0);
    S.E1 = dexpi_rev(r1);
    S.rev0 = r0.v;
    S.drev0[0] = r0.d[0];
    S.drev0[1] = r0.d[1];
    return (int)kc;
}

__device__ __forceinline__ void fresnel_fg_dual(Dn<2> av, Dn<2> &f, Dn<2> &g) {
    if (av.v > 6.0) {
        f = drcp(kPi * av);
        g = dconst<2>(0.0);
    } else {
        Dn<2> a2 = av * av;
        f = (1.0 + 0.926 * av) * drcp((2.0 + 1.792 * av) + 3.104 * a2);
        g = drcp(((2.0 + 4.142 * av) + 3.492 * a2) + 6.670 * (a2 * av));
    }
}

__device__ inline CDn<2> bin_dual(const SpecD &S, int j) {
    const Dn<2> xj = S.x + (double)(-j);
    const Dn<2> xj1 = xj + S.beta;
    if (xj.v > S.r6 || xj1.v < -S.r6) {
        // asymptotic Fresnel on both edges, no crossing: h = i Q (E0 / xj - E1 / xj1)
        const Dn<2> a = drcp(xj), b = drcp(xj1);
        const Dn<2> re = S.E0.re * a - S.E1.re * b;
        const Dn<2> im = S.E0.im * a - S.E1.im * b;
        return {-(S.Q * im), S.Q * re};
    }
    const Dn<2> v0 = S.s * xj, v1 = S.s * xj1;
    const double sg0 = v0.v > 0.0 ? 1.0 : (v0.v < 0.0 ? -1.0 : 0.0);
    const double sg1 = v1.v > 0.0 ? 1.0 : (v1.v < 0.0 ? -1.0 : 0.0);
    Dn<2> f0, g0, f1, g1;
    fresnel_fg_dual(v0 * (sg0 < 0.0 ? -1.0 : 1.0), f0, g0);
    fresnel_fg_dual(v1 * (sg1 < 0.0 ? -1.0 : 1.0), f1, g1);
    const CDn<2> t0 = cdmul(CDn<2>{g0 * sg0, f0 * sg0}, S.E0);
    const CDn<2> t1 = cdmul(CDn<2>{g1 * sg1, f1 * sg1}, S.E1);
    CDn<2> h = cdsub(t0, t1);
    const double ds = sg1 - sg0;
    if (ds != 0.0) {
        // stationary-phase term e^{2 pi i (rev0 - xj^2 / (2 beta))}
        const Dn<2> q = (xj * xj) * S.hib;
        Dn<2> rv;
        rv.v = frac_rev(S.rev0 - q.v);
        rv.d[0] = S.drev0[0] - q.d[0];
        rv.d[1] = S.drev0[1] - q.d[1];
        const CDn<2> e = dexpi_rev(rv);
        const double hh = 0.5 * ds;
        h.re = h.re + hh * (e.re - e.im);
        h.im = h.im + hh * (e.re + e.im);
    }
    return cdscale(h, S.P);
}

// ------------------------------------------------------------------ kernel
struct VjpArgs {
    int M, K, Nt, C;
    double dT, df, fnyq;
    const void *pix;
    int layout;  // 0 layer-major, 1 tranche-major, 2 layer-major with interleaved channels
    const float *layer_scale;
    const double *inv_asd, *tranche_w, *geo, *u_scale;
    const float *rho;  // [K][Nt] per-pixel weight factor (general per-tranche PSD), else NULL
    int64_t n;
    const double *mc, *eta, *f0, *ct, *phi, *psi, *ci;
    const int32_t *nseg;
    const int64_t *seg_offset;
    const double *seg_zn, *g_stat, *g_seg;
    double *g_params;
    uint32_t *counter;  // work counter: each wave takes its next template with one atomic
};

__device__ __forceinline__ double wave_sum_f64(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

template <int C, class PixT>
__global__ __launch_bounds__(256) void k_vjp_wave(VjpArgs a) {
    extern __shared__ unsigned char smem_raw[];
    const int KP = a.K + 2 * kHalfBins;
    double *u_pad = reinterpret_cast<double *>(smem_raw);
    const double u_mul = a.u_scale[0];
    const int kmax = a.M / 2 - 1;
    for (int q = threadIdx.x; q < KP; q += blockDim.x) {
        const int k = q - kHalfBins;
        u_pad[q] = (k >= 1 && k <= kmax) ? a.inv_asd[k] * u_mul : 0.0;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63;
    for (;;) {
        // dynamic work fetch, as in the statistic kernel: one atomic per wave on a uniform address
        const uint32_t mine = atomicAdd(a.counter, lane == 0 ? 1u : 0u);
        const int64_t i = (int64_t)__builtin_amdgcn_readfirstlane(mine);
        if (i >= a.n) break;
        double gr[5] = {0, 0, 0, 0, 0};
        const bool ok = params_valid(a.mc[i], a.eta[i], a.f0[i], a.ct[i], a.ci[i]);
        if (ok) {
            const int ns = a.nseg[i];
            const int64_t off = a.seg_offset[i];
            const double gs = a.g_stat ? a.g_stat[i] : 0.0;
            Track T;
            track_init(T, a.mc[i], a.eta[i], a.f0[i]);
            const TrackTan TT = track_tangents(T, a.f0[i]);
            SkyD S;
            sky_dual(S, a.ct[i], a.phi[i], a.psi[i], a.ci[i]);
            int m_end = a.Nt;
            for (int m0 = 0; m0 < m_end; m0 += 64) {
                const int m = m0 + lane;
                const bool inr = m < a.Nt;
                double Phi = 0.0, f = 0.0, fdot = 0.0;
                const int code = inr ? track_step(T, (double)m * a.dT, a.dT, a.df, a.fnyq, Phi, f, fdot) : 0;
                const uint64_t viol = __ballot(code != 0);
                int lim = a.Nt;
                if (viol) {
                    lim = m0 + __builtin_amdgcn_readfirstlane(__ffsll((unsigned long long)viol) - 1);
                    m_end = lim;
                }
                const bool active = inr && m < lim;
                const double wm = active ? a.tranche_w[m] : 0.0;
                if (active && wm != 0.0) {
                    // adjoint coefficients of this tranche's segment
                    const int sn = (int)(((int64_t)m * ns) / a.Nt);
                    const int64_t o = off + sn;
                    const double zr = a.seg_zn[3 * o], zi = a.seg_zn[3 * o + 1], Nn = a.seg_zn[3 * o + 2];
                    const double g = gs + (a.g_seg ? a.g_seg[o] : 0.0);
                    double ar = 0.0, ai = 0.0, b = 0.0;
                    if (Nn > 0.0 && g != 0.0) {
                        const double iN = 1.0 / Nn;
                        ar = 4.0 * g * zr * iN;
                        ai = -4.0 * g * zi * iN;
                        b = 4.0 * g * (zr * zr + zi * zi) * iN * iN;
                    }
                    if (ar != 0.0 || ai != 0.0 || b != 0.0) {
                        const int m_ref = (int)(((int64_t)sn * a.Nt + ns - 1) / ns);
                        double dref[2];
                        dphi_at(T, TT, (double)m_ref * a.dT, dref);
                        const TrackDual TD = track_dual(T, TT, (double)m * a.dT, f);
                        SpecD sp;
                        const int kc = spec_dual(sp, Phi, f, fdot, TD, dref, a.dT);
                        // bin sums
                        double S1r[C], S1i[C], Ur[C][2], Ui[C][2];
                        double S2 = 0.0, Vr[2] = {0, 0}, Vi[2] = {0, 0};
#pragma unroll
                        for (int c = 0; c < C; ++c) {
                            S1r[c] = S1i[c] = 0.0;
                            Ur[c][0] = Ur[c][1] = Ui[c][0] = Ui[c][1] = 0.0;
                        }
                        for (int j = -kHalfBins; j <= kHalfBins; ++j) {
                            const int k = kc + j;
                            if (k < 1 || k > kmax) continue;
                            double u = u_pad[k + kHalfBins];
                            if (a.rho) u *= (double)a.rho[(size_t)k * a.Nt + m];
                            CDn<2> H = bin_dual(sp, j);
                            H = cdscale(H, u);
                            const double hr = H.re.v, hi = H.im.v;
                            S2 += hr * hr + hi * hi;
#pragma unroll
                            for (int p = 0; p < 2; ++p) {
                                Vr[p] += hr * H.re.d[p] + hi * H.im.d[p];
                                Vi[p] += hr * H.im.d[p] - hi * H.re.d[p];
                            }
#pragma unroll
                            for (int c = 0; c < C; ++c) {
                                const size_t idx = a.layout == 0 ? ((size_t)c * a.K + k) * a.Nt + m
                                                   : (a.layout == 1 ? ((size_t)c * a.Nt + m) * a.K + k
                                                                    : ((size_t)k * a.Nt + m) * C + c);
                                cx<typename PixTraits<PixT>::R> dv = PixTraits<PixT>::load(a.pix, idx);
                                double dr = (double)dv.re, di = (double)dv.im;
                                if constexpr (PixTraits<PixT>::scaled) {
                                    const double sc = (double)a.layer_scale[c * a.K + k];
                                    dr *= sc;
                                    di *= sc;
                                }
                                // conj(D) x
                                S1r[c] += dr * hr + di * hi;
                                S1i[c] += dr * hi - di * hr;
#pragma unroll
                                for (int p = 0; p < 2; ++p) {
                                    Ur[c][p] += dr * H.re.d[p] + di * H.im.d[p];
                                    Ui[c][p] += dr * H.im.d[p] - di * H.re.d[p];
                                }
                            }
                        }
                        // tranche weight: H carries w_m
                        const double w2 = wm * wm;
                        S2 *= w2;
#pragma unroll
                        for (int p = 0; p < 2; ++p) {
                            Vr[p] *= w2;
                            Vi[p] *= w2;
                        }
                        CDn<4> Tc[3];
                        double gm[kGeoRows];
                        load_geo(a.geo, m, a.Nt, gm);
                        transfer_ae_dual<(C == 3)>(S, gm, f, Tc[0], Tc[1], Tc[2]);
#pragma unroll
                        for (int c = 0; c < C; ++c) {
                            const double tr = Tc[c].re.v, ti = Tc[c].im.v;
                            // G_c = a S1_c - b conj(T_c) S2
                            const double s1r = S1r[c] * wm, s1i = S1i[c] * wm;
                            const double Gr = (ar * s1r - ai * s1i) - b * tr * S2;
                            const double Gi = (ar * s1i + ai * s1r) + b * ti * S2;
                            // Re(dT/dq G) for the response slots
                            double rg[4];
#pragma unroll
                            for (int q = 0; q < 4; ++q) rg[q] = Tc[c].re.d[q] * Gr - Tc[c].im.d[q] * Gi;
#pragma unroll
                            for (int p = 0; p < 2; ++p) {
                                const double ur = Ur[c][p] * wm, ui = Ui[c][p] * wm;
                                // J = a U - b conj(T) V
                                const double Jr = (ar * ur - ai * ui) - b * (tr * Vr[p] + ti * Vi[p]);
                                const double Ji = (ar * ui + ai * ur) - b * (tr * Vi[p] - ti * Vr[p]);
                                gr[p] += rg[0] * TD.df[p] + (tr * Jr - ti * Ji);
                            }
                            gr[2] += rg[1];
                            gr[3] += rg[2];
                            gr[4] += rg[3];
                        }
                    }
                }
                if (viol) break;
            }
        }
#pragma unroll
        for (int p = 0; p < 5; ++p) gr[p] = wave_sum_f64(gr[p]);
        if (lane == 0) {
            // ln Mc, f0, cos theta, phi, psi
#pragma unroll
            for (int p = 0; p < 5; ++p) a.g_params[5 * i + p] = gr[p];
        }
    }
}

__global__ void k_vjp_zero(uint32_t *counter) {
    if (threadIdx.x == 0) counter[0] = 0u;
}

template <int C, class PixT>
static hipError_t launch_vjp_t(const VjpArgs &a, int n_groups, int block_waves, hipStream_t st) {
    const size_t shmem = sizeof(double) * ((size_t)a.K + 2 * kHalfBins);
    hipLaunchKernelGGL((k_vjp_wave<C, PixT>), dim3(n_groups), dim3(64 * block_waves), shmem, st, a);
    return hipGetLastError();
}

template <int C>
static hipError_t dispatch_vjp(const VjpArgs &a, int dtype, int n_groups, int block_waves, hipStream_t st) {
    switch (dtype) {
        case 0: return launch_vjp_t<C, double>(a, n_groups, block_waves, st);
        case 1: return launch_vjp_t<C, float>(a, n_groups, block_waves, st);
        case 2: return launch_vjp_t<C, __hip_bfloat16>(a, n_groups, block_waves, st);
        case 3: return launch_vjp_t<C, __half>(a, n_groups, block_waves, st);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_vjp(const VjpLaunch &V, hipStream_t st) {
    const StatLaunch &L = V.s;
    if (L.n == 0) return hipSuccess;
    VjpArgs a;
    a.M = L.M;
    a.K = L.M / 2 + 1;
    a.Nt = L.Nt;
    a.C = L.C;
    a.dT = (double)L.M * L.dt;
    a.df = 1.0 / a.dT;
    a.fnyq = 0.5 / L.dt;
    a.pix = L.pix;
    a.layout = L.layout;
    a.layer_scale = L.layer_scale;
    a.inv_asd = L.inv_asd;
    a.tranche_w = L.tranche_w;
    a.geo = L.geo;
    a.u_scale = L.u_scale;
    a.rho = L.rho;
    a.n = L.n;
    a.mc = L.mc;
    a.eta = L.eta;
    a.f0 = L.f0;
    a.ct = L.ct;
    a.phi = L.phi;
    a.psi = L.psi;
    a.ci = L.ci;
    a.nseg = L.nseg;
    a.seg_offset = L.seg_offset;
    a.seg_zn = V.seg_zn;
    a.g_stat = V.g_stat;
    a.g_seg = V.g_seg;
    a.g_params = V.g_params;
    a.counter = L.counter;
    const int bw = L.block_waves;
    int64_t groups = (L.n + bw - 1) / bw;
    if (groups > (int64_t)L.n_groups) groups = L.n_groups;
    hipLaunchKernelGGL(k_vjp_zero, dim3(1), dim3(64), 0, st, a.counter);
    if (L.C == 3) return dispatch_vjp<3>(a, L.pix_dtype, (int)groups, bw, st);
    return L.C == 1 ? dispatch_vjp<1>(a, L.pix_dtype, (int)groups, bw, st)
                    : dispatch_vjp<2>(a, L.pix_dtype, (int)groups, bw, st);
}

}  // namespace tfsc
