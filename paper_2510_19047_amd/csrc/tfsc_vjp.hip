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
#include "tfsc_stat_common.hpp"  // wave_uniform, dpp_sum_f64

// The tangent arithmetic below contracts multiply-adds into FMAs.  The FP64 track that fixes
// the integer structure (track_step, from tfsc_device.hpp, included above) is not affected.
#pragma clang fp contract(fast)

namespace tfsc {

// ------------------------------------------------------------------ dual numbers
// Dn<N, R>: a value and N tangents in arithmetic R (double, or float for the FP32 form).  Scalars
// mixed with a dual number take its type (nd_t keeps them out of template deduction).
template <class T>
struct nodeduce {
    using type = T;
};
template <class T>
using nd_t = typename nodeduce<T>::type;

template <int N, class R = double>
struct Dn {
    R v;
    R d[N];
};

template <int N, class R>
__device__ __forceinline__ Dn<N, R> dconst(nd_t<R> v) {
    Dn<N, R> r;
    r.v = v;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = (R)0;
    return r;
}
template <int N, class R>
__device__ __forceinline__ Dn<N, R> operator+(Dn<N, R> a, Dn<N, R> b) {
    Dn<N, R> r;
    r.v = a.v + b.v;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = a.d[i] + b.d[i];
    return r;
}
template <int N, class R>
__device__ __forceinline__ Dn<N, R> operator-(Dn<N, R> a, Dn<N, R> b) {
    Dn<N, R> r;
    r.v = a.v - b.v;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = a.d[i] - b.d[i];
    return r;
}
template <int N, class R>
__device__ __forceinline__ Dn<N, R> operator-(Dn<N, R> a) {
    Dn<N, R> r;
    r.v = -a.v;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = -a.d[i];
    return r;
}
template <int N, class R>
__device__ __forceinline__ Dn<N, R> operator*(Dn<N, R> a, Dn<N, R> b) {
    Dn<N, R> r;
    r.v = a.v * b.v;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i];
    return r;
}
template <int N, class R>
__device__ __forceinline__ Dn<N, R> operator*(Dn<N, R> a, nd_t<R> s) {
    Dn<N, R> r;
    r.v = a.v * s;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * s;
    return r;
}
template <int N, class R>
__device__ __forceinline__ Dn<N, R> operator*(nd_t<R> s, Dn<N, R> a) {
    return a * s;
}
template <int N, class R>
__device__ __forceinline__ Dn<N, R> operator+(Dn<N, R> a, nd_t<R> s) {
    a.v += s;
    return a;
}
template <int N, class R>
__device__ __forceinline__ Dn<N, R> operator+(nd_t<R> s, Dn<N, R> a) {
    a.v += s;
    return a;
}
template <int N, class R>
__device__ __forceinline__ Dn<N, R> operator-(nd_t<R> s, Dn<N, R> a) {
    return (-a) + s;
}
template <int N, class R>
__device__ __forceinline__ Dn<N, R> drcp(Dn<N, R> a) {
    const R r = rcp(a.v), r2 = -r * r;
    Dn<N, R> o;
    o.v = r;
#pragma unroll
    for (int i = 0; i < N; ++i) o.d[i] = a.d[i] * r2;
    return o;
}
__device__ __forceinline__ double vsqrt(double x) { return sqrt(x); }
__device__ __forceinline__ float vsqrt(float x) { return sqrtf(x); }
__device__ __forceinline__ double half_rcp(double s) { return 0.5 / s; }
__device__ __forceinline__ float half_rcp(float s) { return 0.5f * rcp(s); }
template <int N, class R>
__device__ __forceinline__ Dn<N, R> dsqrt(Dn<N, R> a) {
    const R s = vsqrt(a.v), h = half_rcp(s);
    Dn<N, R> o;
    o.v = s;
#pragma unroll
    for (int i = 0; i < N; ++i) o.d[i] = a.d[i] * h;
    return o;
}
// sine and cosine of 2 pi r for r in revolutions (|r| <= 1/2)
__device__ __forceinline__ void sincos_rev(double r, double &s, double &c) { sincospi(2.0 * r, &s, &c); }
__device__ __forceinline__ void sincos_rev(float r, float &s, float &c) {
    s = __builtin_amdgcn_sinf(r);
    c = __builtin_amdgcn_cosf(r);
}
// sin(2 pi r) with its tangent; in FP32 the value is taken of the argument folded into
// [-1/4, 1/4] (exact in FP32) so that it keeps its relative precision near the zeros r = +-1/2
template <int N, class R>
__device__ __forceinline__ Dn<N, R> dsin_rev(Dn<N, R> r) {
    R s, c;
    sincos_rev(r.v, s, c);
    if constexpr (sizeof(R) == 4) {
        const float rf = r.v > 0.25f ? 0.5f - r.v : (r.v < -0.25f ? -0.5f - r.v : r.v);
        s = sin_rev_accurate(rf);
    }
    Dn<N, R> o;
    o.v = s;
#pragma unroll
    for (int i = 0; i < N; ++i) o.d[i] = (R)kTwoPi * c * r.d[i];
    return o;
}
// sin(x)/x and its derivative (cos x - sin x / x) / x, for x >= 0
__device__ __forceinline__ void sinc_d(double x, double &v, double &dv) {
    if (fabs(x) < 1e-4) {
        v = 1.0 - x * x * (1.0 / 6.0);
        dv = -x * (1.0 / 3.0);
    } else {
        double s, c;
        sincos(x, &s, &c);
        v = s / x;
        dv = (c - v) / x;
    }
}
__device__ __forceinline__ void sinc_d(float x, float &v, float &dv) {
    if (x < 0.5f) {
        // Taylor series of sin x / x through x^8 and of its derivative through x^7 (first omitted
        // terms below 6e-10 and 1.3e-10 at x = 1/2), free of the cancellation in (cos x - v) / x
        const float x2 = x * x;
        v = 1.0f - x2 * (1.0f / 6.0f - x2 * (1.0f / 120.0f - x2 * (1.0f / 5040.0f - x2 * (1.0f / 362880.0f))));
        dv = -x * (1.0f / 3.0f - x2 * (1.0f / 30.0f - x2 * (1.0f / 840.0f - x2 * (1.0f / 45360.0f))));
    } else {
        const float r = x * (float)(1.0 / kTwoPi), ir = rcp(x);
        v = __builtin_amdgcn_sinf(r) * ir;
        dv = (__builtin_amdgcn_cosf(r) - v) * ir;
    }
}
template <int N, class R>
__device__ __forceinline__ Dn<N, R> dsinc(Dn<N, R> x) {
    R v, dv;
    sinc_d(x.v, v, dv);
    Dn<N, R> o;
    o.v = v;
#pragma unroll
    for (int i = 0; i < N; ++i) o.d[i] = dv * x.d[i];
    return o;
}

template <int N, class R = double>
struct CDn {
    Dn<N, R> re, im;
};
template <int N, class R>
__device__ __forceinline__ CDn<N, R> cdmul(CDn<N, R> a, CDn<N, R> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <int N, class R>
__device__ __forceinline__ CDn<N, R> cdadd(CDn<N, R> a, CDn<N, R> b) {
    return {a.re + b.re, a.im + b.im};
}
template <int N, class R>
__device__ __forceinline__ CDn<N, R> cdsub(CDn<N, R> a, CDn<N, R> b) {
    return {a.re - b.re, a.im - b.im};
}
template <int N, class R>
__device__ __forceinline__ CDn<N, R> cdscale(CDn<N, R> a, Dn<N, R> s) {
    return {a.re * s, a.im * s};
}
template <int N, class R>
__device__ __forceinline__ CDn<N, R> cdscale(CDn<N, R> a, nd_t<R> s) {
    return {a.re * s, a.im * s};
}
// e^{2 pi i r} for r in revolutions (|r| <= 1/2)
template <int N, class R>
__device__ __forceinline__ CDn<N, R> dexpi_rev(Dn<N, R> r) {
    R s, c;
    sincos_rev(r.v, s, c);
    CDn<N, R> o;
    o.re.v = c;
    o.im.v = s;
#pragma unroll
    for (int i = 0; i < N; ++i) {
        o.re.d[i] = -(R)kTwoPi * s * r.d[i];
        o.im.d[i] = (R)kTwoPi * c * r.d[i];
    }
    return o;
}
template <class R, int N>
__device__ __forceinline__ Dn<N, R> to_r(const Dn<N, double> &a) {
    Dn<N, R> o;
    o.v = (R)a.v;
#pragma unroll
    for (int i = 0; i < N; ++i) o.d[i] = (R)a.d[i];
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

// Phase, frequency and chirp tangents at t < t_c.  s = 1/theta comes from the forward's track_at (its theta is
// rcp_rn(s)); the per-template divisors enter through their reciprocals and theta^-6 as s^6, since the
// tangents need no correctly rounded quotients.
struct TrackDual {
    double dPhi[2], df[2], dfdot[2];
};

__device__ inline TrackDual track_dual(const Track &T, const TrackTan &G, double t, double f, double s) {
    const double tau = T.tc - t;
    const double itau = rcp_rn(tau);
    const double th = rcp_rn(s);
    const double th2 = th * th, th3 = th2 * th, th4 = th2 * th2, th5 = th4 * th, th9 = th5 * th4;
    const double s2 = s * s, s6 = (s2 * s2) * s2;  // theta^-6
    const double dPf = ((3.0 + (5.0 * T.a2) * th2) + (6.0 * T.a3) * th3) + (7.0 * T.a4) * th4;
    const double ddPf = ((10.0 * T.a2) * th + (18.0 * T.a3) * th2) + (28.0 * T.a4) * th3;
    const double dfdth = (th2 * T.rc8) * dPf;
    const double dthdt = (T.eta * th9) * T.r40M;
    const double Pp = ((1.0 + T.b2 * th2) + T.b3 * th3) + T.b4 * th4;
    const double dPp = ((2.0 * T.b2) * th + (3.0 * T.b3) * th2) + (4.0 * T.b4) * th3;
    const double dPhidth = (2.0 * T.reta) * (5.0 * Pp - th * dPp) * s6;
    TrackDual D;
#pragma unroll
    for (int p = 0; p < 2; ++p) {
        const double mu = G.mu[p];
        const double dth = -0.125 * th * (G.dtc[p] * itau - mu);
        D.df[p] = dfdth * dth - f * mu;
        const double d_dfdth = ((2.0 * th * dPf + th2 * ddPf) * T.rc8) * dth - dfdth * mu;
        const double d_dthdt = dthdt * (9.0 * dth / th - mu);
        D.dfdot[p] = d_dfdth * dthdt + dfdth * d_dthdt;
        D.dPhi[p] = dPhidth * dth;
    }
    return D;
}

__device__ inline void dphi_at(const Track &T, const TrackTan &G, double t, double out[2]) {
    const double tau = T.tc - t;
    const double itau = rcp_rn(tau);
    const double s = sqrt_pos(sqrt_pos(sqrt_pos((T.eta * tau) * T.r5M)));
    const double th = rcp_rn(s);
    const double th2 = th * th, th3 = th2 * th, th4 = th2 * th2;
    const double s2 = s * s, s6 = (s2 * s2) * s2;  // theta^-6
    const double Pp = ((1.0 + T.b2 * th2) + T.b3 * th3) + T.b4 * th4;
    const double dPp = ((2.0 * T.b2) * th + (3.0 * T.b3) * th2) + (4.0 * T.b4) * th3;
    const double dPhidth = (2.0 * T.reta) * (5.0 * Pp - th * dPp) * s6;
#pragma unroll
    for (int p = 0; p < 2; ++p) out[p] = dPhidth * (-0.125 * th * (G.dtc[p] * itau - G.mu[p]));
}

// ------------------------------------------------------------------ response tangents
// Tangent slots: 0 = f, 1 = cos theta, 2 = phi, 3 = psi.  Same formulas as transfer_ae.  The
// sky constants are formed in FP64 and rounded to R; kv keeps the FP64 propagation direction,
// from which the light-travel phases are formed in FP64 in both arithmetics.
template <class R>
struct SkyD {
    Dn<4, R> k[3], u[3], v[3], c2, s2;
    R ap, ci;
    double kv[3];
};

template <class R>
__device__ inline void sky_dual(SkyD<R> &S, double ct, double phi, double psi, double ci) {
    Dn<4> c = dconst<4, double>(ct);
    c.d[1] = 1.0;
    double sp, cp, s2, c2;
    sincos(phi, &sp, &cp);
    sincos(2.0 * psi, &s2, &c2);
    Dn<4> Sp = dconst<4, double>(sp), Cp = dconst<4, double>(cp);
    Sp.d[2] = cp;
    Cp.d[2] = -sp;
    Dn<4> st = dsqrt(1.0 - c * c);
    const Dn<4> k[3] = {-(st * Cp), -(st * Sp), -c};
    const Dn<4> u[3] = {c * Cp, c * Sp, -st};
    const Dn<4> v[3] = {Sp, -Cp, dconst<4, double>(0.0)};
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        S.k[i] = to_r<R>(k[i]);
        S.u[i] = to_r<R>(u[i]);
        S.v[i] = to_r<R>(v[i]);
        S.kv[i] = k[i].v;
    }
    S.c2 = dconst<4, R>((R)c2);
    S.s2 = dconst<4, R>((R)s2);
    S.c2.d[3] = (R)(-2.0 * s2);
    S.s2.d[3] = (R)(2.0 * c2);
    S.ap = (R)((1.0 + ci * ci) / 2.0);
    S.ci = (R)ci;
}

template <bool WITH_T, class R>
__device__ inline void transfer_ae_dual(const SkyD<R> &S, const double (&g)[kGeoRows], double f, CDn<4, R> &TA,
                                        CDn<4, R> &TE, CDn<4, R> &TT) {
    const double L = kArmM / kClight;
    Dn<4, R> F = dconst<4, R>((R)f);
    F.d[0] = (R)1;
    Dn<4, R> kp[3];
    double kpv[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        kp[i] = S.k[0] * (R)g[3 * i] + S.k[1] * (R)g[3 * i + 1] + S.k[2] * (R)g[3 * i + 2];
        kpv[i] = S.kv[0] * g[3 * i] + S.kv[1] * g[3 * i + 1] + S.kv[2] * g[3 * i + 2];
    }
    const Dn<4, R> pfL = F * (R)(kPi * L);
    CDn<4, R> Gd[3], Gr[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int s = a, r = (a + 1) % 3;
        const R n0 = (R)g[9 + 3 * a + 0];
        const R n1 = (R)g[9 + 3 * a + 1];
        const R n2 = (R)g[9 + 3 * a + 2];
        Dn<4, R> kn = S.k[0] * n0 + S.k[1] * n1 + S.k[2] * n2;
        Dn<4, R> nu = S.u[0] * n0 + S.u[1] * n1 + S.u[2] * n2;
        Dn<4, R> nv = S.v[0] * n0 + S.v[1] * n1 + S.v[2] * n2;
        Dn<4, R> xp0 = nu * nu - nv * nv, xx0 = 2.0 * (nu * nv);
        Dn<4, R> xp = S.c2 * xp0 + S.s2 * xx0;
        Dn<4, R> xx = S.s2 * (-xp0) + S.c2 * xx0;
        CDn<4, R> amp = {xp * S.ap, xx * (-S.ci)};
        // -pi f (L + k.(p_s + p_r)) in revolutions: value reduced in FP64, tangents in R
        const double ksv = (kpv[s] + kpv[r]) + L;
        const double fh = f * (-0.5);
        Dn<4, R> rev;
        rev.v = (R)frac_rev(fh * ksv);
#pragma unroll
        for (int q = 0; q < 4; ++q) rev.d[q] = (R)fh * (kp[s].d[q] + kp[r].d[q]);
        rev.d[0] += (R)(-0.5 * ksv);
        CDn<4, R> Ea = cdmul(dexpi_rev(rev), amp);
        CDn<4, R> B = {pfL * Ea.im, -(pfL * Ea.re)};
        Gd[a] = cdscale(B, dsinc(pfL * (1.0 - kn)));
        Gr[a] = cdscale(B, dsinc(pfL * (1.0 + kn)));
    }
    const CDn<4, R> G01 = Gd[0], G10 = Gr[0], G12 = Gd[1], G21 = Gr[1], G20 = Gd[2], G02 = Gr[2];
    // 1 - D^2 = 2 i sin(2 pi f L) D, D = e^{-2 pi i f L}
    Dn<4, R> rl = dconst<4, R>((R)frac_rev(f * L));
    rl.d[0] = (R)L;
    const CDn<4, R> D = dexpi_rev(-rl);
    const Dn<4, R> s2 = dsin_rev(rl);
    const CDn<4, R> om = {(-2.0) * (s2 * D.im), 2.0 * (s2 * D.re)};
    const CDn<4, R> TX = cdmul(om, cdsub(cdadd(G20, cdmul(D, G02)), cdadd(G10, cdmul(D, G01))));
    const CDn<4, R> TY = cdmul(om, cdsub(cdadd(G01, cdmul(D, G10)), cdadd(G21, cdmul(D, G12))));
    const CDn<4, R> TZ = cdmul(om, cdsub(cdadd(G12, cdmul(D, G21)), cdadd(G02, cdmul(D, G20))));
    const double is2 = 0.70710678118654752440, is6 = 0.40824829046386301637;
    TA = cdscale(cdsub(TZ, TX), is2);
    TE = cdscale(cdadd(cdsub(TX, cdscale(TY, 2.0)), TZ), is6);
    if constexpr (WITH_T) TT = cdscale(cdadd(cdadd(TX, TY), TZ), 0.57735026918962576451);  // (X + Y + Z) / sqrt3
}

// ------------------------------------------------------------------ spectrum tangents
// Tangent slots: 0 = ln Mc, 1 = f0.  Bin-relative Fresnel form as in tranche_spectrum_bin; the
// bin index, offset, phases and the Fresnel branch ranges come from FP64 as in tranche_setup,
// so the integer structure is the forward's.
template <class R>
struct SpecD {
    Dn<2, R> x, beta, s, P, Q, hib;
    CDn<2, R> E0, E1;
    double rev0;
    R drev0[2];
    int j0lo, j0hi, j1lo, j1hi;
};

template <class R>
__device__ inline int spec_dual(SpecD<R> &S, double Phi, double f, double fdot, const TrackDual &D,
                                const double dref[2], double dT) {
    const double fT = f * dT;
    const double kc = ceil(fT);
    const double x = fT - kc, beta = (fdot * dT) * dT;
    S.x = dconst<2, R>((R)x);
    S.beta = dconst<2, R>((R)beta);
    Dn<2, R> A, Fd = dconst<2, R>((R)fdot);
    if constexpr (sizeof(R) == 8)
        A.v = pow(f, 2.0 / 3.0);
    else
        A.v = __builtin_amdgcn_exp2f(__builtin_amdgcn_logf((float)f) * (2.0f / 3.0f));
    const R dlnA = (R)(2.0 / 3.0) * (A.v / (R)f);
    const double rev0 = phase_to_rev(Phi);
    Dn<2, R> r0 = dconst<2, R>((R)rev0);
#pragma unroll
    for (int p = 0; p < 2; ++p) {
        S.x.d[p] = (R)(dT * D.df[p]);
        S.beta.d[p] = (R)((dT * dT) * D.dfdot[p]);
        A.d[p] = dlnA * (R)D.df[p];
        Fd.d[p] = (R)D.dfdot[p];
        r0.d[p] = (R)((D.dPhi[p] - dref[p]) * (1.0 / kTwoPi));
    }
    S.s = dsqrt(2.0 * drcp(S.beta));
    S.P = A * drcp(dsqrt(2.0 * Fd));
    S.Q = A * (dT / kTwoPi);
    S.hib = 0.5 * drcp(S.beta);
    {
        const double r6 = sqrt(18.0 * beta);  // 6 / s: |v| <= 6 takes the paper's rational forms
        S.j0lo = (int)ceil(x - r6);
        S.j0hi = (int)floor(x + r6);
        S.j1lo = (int)ceil((x + beta) - r6);
        S.j1hi = (int)floor((x + beta) + r6);
    }
    Dn<2, R> r1 = r0 + S.x + 0.5 * S.beta;
    r1.v = (R)frac_rev(rev0 + x + 0.5 * beta);
    S.E0 = dexpi_rev(r0);
    S.E1 = dexpi_rev(r1);
    S.rev0 = rev0;
    S.drev0[0] = r0.d[0];
    S.drev0[1] = r0.d[1];
    return (int)kc;
}

template <class R>
__device__ __forceinline__ void fresnel_fg_dual(Dn<2, R> av, bool rational, Dn<2, R> &f, Dn<2, R> &g) {
    if (!rational) {
        f = drcp(kPi * av);
        g = dconst<2, R>((R)0);
    } else {
        Dn<2, R> a2 = av * av;
        f = (1.0 + 0.926 * av) * drcp((2.0 + 1.792 * av) + 3.104 * a2);
        g = drcp(((2.0 + 4.142 * av) + 3.492 * a2) + 6.670 * (a2 * av));
    }
}

template <class R>
__device__ inline CDn<2, R> bin_dual(const SpecD<R> &S, int j) {
    const Dn<2, R> xj = S.x + (R)(-j);
    const Dn<2, R> xj1 = xj + S.beta;
    if (j < S.j0lo || j > S.j1hi) {
        // asymptotic Fresnel on both edges, no crossing: h = i Q (E0 / xj - E1 / xj1)
        const Dn<2, R> a = drcp(xj), b = drcp(xj1);
        const Dn<2, R> re = S.E0.re * a - S.E1.re * b;
        const Dn<2, R> im = S.E0.im * a - S.E1.im * b;
        return {-(S.Q * im), S.Q * re};
    }
    const Dn<2, R> v0 = S.s * xj, v1 = S.s * xj1;
    const R sg0 = v0.v > (R)0 ? (R)1 : (v0.v < (R)0 ? (R)-1 : (R)0);
    const R sg1 = v1.v > (R)0 ? (R)1 : (v1.v < (R)0 ? (R)-1 : (R)0);
    Dn<2, R> f0, g0, f1, g1;
    fresnel_fg_dual(v0 * (sg0 < (R)0 ? (R)-1 : (R)1), j >= S.j0lo && j <= S.j0hi, f0, g0);
    fresnel_fg_dual(v1 * (sg1 < (R)0 ? (R)-1 : (R)1), j >= S.j1lo && j <= S.j1hi, f1, g1);
    const CDn<2, R> t0 = cdmul(CDn<2, R>{g0 * sg0, f0 * sg0}, S.E0);
    const CDn<2, R> t1 = cdmul(CDn<2, R>{g1 * sg1, f1 * sg1}, S.E1);
    CDn<2, R> h = cdsub(t0, t1);
    const R ds = sg1 - sg0;
    if (ds != (R)0) {
        // stationary-phase term e^{2 pi i (rev0 - xj^2 / (2 beta))}
        const Dn<2, R> q = (xj * xj) * S.hib;
        Dn<2, R> rv;
        rv.v = (R)frac_rev(S.rev0 - (double)q.v);
        rv.d[0] = S.drev0[0] - q.d[0];
        rv.d[1] = S.drev0[1] - q.d[1];
        const CDn<2, R> e = dexpi_rev(rv);
        const R hh = (R)0.5 * ds;
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

// R = double: the FP64 form; R = float: FP32 spectra, response, pixel sums and tangents (the
// track, its tangents, the phases and every integer decision stay FP64, as in the FP32 forward).
// The FP32 form holds half the registers and runs two waves per SIMD.
template <int C, class PixT, class R>
__global__ __launch_bounds__(256, sizeof(R) == 4 ? 2 : 1) void k_vjp_wave(VjpArgs a) {
    extern __shared__ unsigned char smem_raw[];
    const int KP = a.K + 2 * kHalfBins;
    R *u_pad = reinterpret_cast<R *>(smem_raw);
    const double u_mul = a.u_scale[0];
    const int kmax = a.M / 2 - 1;
    for (int q = threadIdx.x; q < KP; q += blockDim.x) {
        const int k = q - kHalfBins;
        u_pad[q] = (R)((k >= 1 && k <= kmax) ? a.inv_asd[k] * u_mul : 0.0);
    }
    __syncthreads();
    const int lane = threadIdx.x & 63;
    for (;;) {
        // dynamic work fetch, as in the statistic kernel: one atomic per wave on a uniform address
        const uint32_t mine = atomicAdd(a.counter, lane == 0 ? 1u : 0u);
        const int64_t i = (int64_t)__builtin_amdgcn_readfirstlane(mine);
        if (i >= a.n) break;
        double gr[5] = {0, 0, 0, 0, 0};
        const double mci = a.mc[i];
        const bool ok = params_valid(mci, a.eta[i], a.f0[i], a.ct[i], a.ci[i]);
        if (ok) {
            const int ns = a.nseg[i];
            const int64_t off = a.seg_offset[i];
            const double gs = a.g_stat ? a.g_stat[i] : 0.0;
            Track T;
            track_init(T, mci, a.eta[i], a.f0[i]);
            wave_uniform(T);
            TrackTan TT = track_tangents(T, a.f0[i]);
#pragma unroll
            for (int p = 0; p < 2; ++p) {
                TT.mu[p] = wave_uniform(TT.mu[p]);
                TT.dtc[p] = wave_uniform(TT.dtc[p]);
            }
            SkyD<R> S;
            sky_dual(S, a.ct[i], a.phi[i], a.psi[i], a.ci[i]);
            int m_end = a.Nt;
            // FP32 form (two waves per SIMD): each chunk's track is evaluated during the previous chunk, beside
            // that chunk's response tangents, so the dependent FP64 chain overlaps the FP32 work.  The FP64 form
            // (one wave per SIMD, at its register limit) evaluates it at the top of its chunk, which measured faster.
            constexpr bool kAhead = sizeof(R) == 4;
            double Phi = 0.0, f = 0.0, fdot = 0.0, s_th = 1.0;
            int code = 0;
            if constexpr (kAhead) {
                code = track_step_lanes(T, (double)(lane < a.Nt ? lane : a.Nt - 1) * a.dT, a.dT, a.df, a.fnyq, Phi, f,
                                        fdot, &s_th);
                code = lane < a.Nt ? code : 0;
            }
            for (int m0 = 0; m0 < m_end; m0 += 64) {
                const int m = m0 + lane;
                const bool inr = m < a.Nt;
                if constexpr (!kAhead) {
                    code = track_step_lanes(T, (double)(inr ? m : a.Nt - 1) * a.dT, a.dT, a.df, a.fnyq, Phi, f, fdot,
                                            &s_th);
                    code = inr ? code : 0;
                }
                const uint64_t viol = __ballot(code != 0);
                int lim = a.Nt;
                if (viol) {
                    lim = m0 + __builtin_amdgcn_readfirstlane(__ffsll((unsigned long long)viol) - 1);
                    m_end = lim;
                }
                const bool active = inr && m < lim;
                const double wm = active ? a.tranche_w[m] : 0.0;
                // adjoint coefficients of this tranche's segment
                double ar = 0.0, ai = 0.0, b = 0.0;
                int sn = 0;
                if (active && wm != 0.0) {
                    sn = (int)(((int64_t)m * ns) / a.Nt);
                    const int64_t o = off + sn;
                    const double zr = a.seg_zn[3 * o], zi = a.seg_zn[3 * o + 1], Nn = a.seg_zn[3 * o + 2];
                    const double g = gs + (a.g_seg ? a.g_seg[o] : 0.0);
                    if (Nn > 0.0 && g != 0.0) {
                        const double iN = 1.0 / Nn;
                        ar = 4.0 * g * zr * iN;
                        ai = -4.0 * g * zi * iN;
                        b = 4.0 * g * (zr * zr + zi * zi) * iN * iN;
                    }
                }
                const bool work = ar != 0.0 || ai != 0.0 || b != 0.0;
                // pixel and spectrum sums of the working lanes
                R S1r[C], S1i[C], Ur[C][2], Ui[C][2];
                R S2 = (R)0, Vr[2] = {(R)0, (R)0}, Vi[2] = {(R)0, (R)0};
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    S1r[c] = S1i[c] = (R)0;
                    Ur[c][0] = Ur[c][1] = Ui[c][0] = Ui[c][1] = (R)0;
                }
                R dfr[2] = {(R)0, (R)0};
                {
                    if (work) {
                        const int m_ref = (int)(((int64_t)sn * a.Nt + ns - 1) / ns);
                        double dref[2];
                        dphi_at(T, TT, (double)m_ref * a.dT, dref);
                        const TrackDual TD = track_dual(T, TT, (double)m * a.dT, f, s_th);
                        dfr[0] = (R)TD.df[0];
                        dfr[1] = (R)TD.df[1];
                        SpecD<R> sp;
                        const int kc = spec_dual(sp, Phi, f, fdot, TD, dref, a.dT);
                        for (int j = -kHalfBins; j <= kHalfBins; ++j) {
                            const int k = kc + j;
                            if (k < 1 || k > kmax) continue;
                            R u = u_pad[k + kHalfBins];
                            if (a.rho) u *= (R)a.rho[(size_t)k * a.Nt + m];
                            CDn<2, R> H = bin_dual(sp, j);
                            H = cdscale(H, u);
                            const R hr = H.re.v, hi = H.im.v;
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
                                R dr = (R)dv.re, di = (R)dv.im;
                                if constexpr (PixTraits<PixT>::scaled) {
                                    const R sc = (R)a.layer_scale[c * a.K + k];
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
                    }
                }
                // this chunk's response tangents and the next chunk's track, for every lane (values of lanes
                // without work are not used; the geometry row is clamped into the table)
                CDn<4, R> Tc[3];
                {
                    double gm[kGeoRows];
                    load_geo(a.geo, inr ? m : a.Nt - 1, a.Nt, gm);
                    transfer_ae_dual<(C == 3)>(S, gm, f, Tc[0], Tc[1], Tc[2]);
                    if constexpr (kAhead) {
                        const int mn = m + 64;
                        int cn = track_step_lanes(T, (double)(mn < a.Nt ? mn : a.Nt - 1) * a.dT, a.dT, a.df, a.fnyq, Phi,
                                                  f, fdot, &s_th);
                        code = mn < a.Nt ? cn : 0;
                    }
                }
                if (work) {
                    {
                        // tranche weight: H carries w_m
                        const R wr = (R)wm, w2 = wr * wr;
                        S2 *= w2;
#pragma unroll
                        for (int p = 0; p < 2; ++p) {
                            Vr[p] *= w2;
                            Vi[p] *= w2;
                        }
                        const R arr = (R)ar, air = (R)ai, br = (R)b;
#pragma unroll
                        for (int c = 0; c < C; ++c) {
                            const R tr = Tc[c].re.v, ti = Tc[c].im.v;
                            // G_c = a S1_c - b conj(T_c) S2
                            const R s1r = S1r[c] * wr, s1i = S1i[c] * wr;
                            const R Gr = (arr * s1r - air * s1i) - br * tr * S2;
                            const R Gi = (arr * s1i + air * s1r) + br * ti * S2;
                            // Re(dT/dq G) for the response slots
                            R rg[4];
#pragma unroll
                            for (int q = 0; q < 4; ++q) rg[q] = Tc[c].re.d[q] * Gr - Tc[c].im.d[q] * Gi;
#pragma unroll
                            for (int p = 0; p < 2; ++p) {
                                const R ur = Ur[c][p] * wr, ui = Ui[c][p] * wr;
                                // J = a U - b conj(T) V
                                const R Jr = (arr * ur - air * ui) - br * (tr * Vr[p] + ti * Vi[p]);
                                const R Ji = (arr * ui + air * ur) - br * (tr * Vi[p] - ti * Vr[p]);
                                gr[p] += (double)(rg[0] * dfr[p] + (tr * Jr - ti * Ji));
                            }
                            gr[2] += (double)rg[1];
                            gr[3] += (double)rg[2];
                            gr[4] += (double)rg[3];
                        }
                    }
                }
                if (viol) break;
            }
        }
#pragma unroll
        for (int p = 0; p < 5; ++p) gr[p] = dpp_sum_f64(gr[p]);
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

template <int C, class PixT, class R>
static hipError_t launch_vjp_t(const VjpArgs &a, int n_groups, int block_waves, hipStream_t st) {
    const size_t shmem = sizeof(R) * ((size_t)a.K + 2 * kHalfBins);
    hipLaunchKernelGGL((k_vjp_wave<C, PixT, R>), dim3(n_groups), dim3(64 * block_waves), shmem, st, a);
    return hipGetLastError();
}

template <int C, class R>
static hipError_t dispatch_vjp(const VjpArgs &a, int dtype, int n_groups, int block_waves, hipStream_t st) {
    switch (dtype) {
        case 0: return launch_vjp_t<C, double, R>(a, n_groups, block_waves, st);
        case 1: return launch_vjp_t<C, float, R>(a, n_groups, block_waves, st);
        case 2: return launch_vjp_t<C, __hip_bfloat16, R>(a, n_groups, block_waves, st);
        case 3: return launch_vjp_t<C, __half, R>(a, n_groups, block_waves, st);
        case 4: return launch_vjp_t<C, int16_t, R>(a, n_groups, block_waves, st);
    }
    return hipErrorInvalidValue;
}

template <class R>
static hipError_t dispatch_vjp_c(const VjpArgs &a, int C, int dtype, int n_groups, int block_waves, hipStream_t st) {
    if (C == 3) return dispatch_vjp<3, R>(a, dtype, n_groups, block_waves, st);
    return C == 1 ? dispatch_vjp<1, R>(a, dtype, n_groups, block_waves, st)
                  : dispatch_vjp<2, R>(a, dtype, n_groups, block_waves, st);
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
    return L.precision == 1 ? dispatch_vjp_c<float>(a, L.C, L.pix_dtype, (int)groups, bw, st)
                            : dispatch_vjp_c<double>(a, L.C, L.pix_dtype, (int)groups, bw, st);
}

}  // namespace tfsc
