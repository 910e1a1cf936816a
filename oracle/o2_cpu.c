/*
 * O2 oracle in plain scalar C (FP64), one OpenMP thread per template.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  It computes exactly
 * what oracle/o2.py computes -- the paper's Fresnel-kernel method written
 * literally -- and exists to time the oracle on host cores and to evaluate
 * large parity samples.  It shares no source with the HIP library.
 *
 * Paper passages: Eq. (Upsilon-seg), Eq. (overlap-n), Eqs. (inner-segment-tf)
 * and (inner-tranche-tf), Eq. (fresnel-ft) with the two Fresnel branches,
 * Eq. (tdi2) (transfer once per tranche), N_F = 21 bins around the bin just
 * above f_nm, Appendix A compactness.  The TaylorT3 track, the response
 * reconstruction and the normalisation are those stated in oracle/track.py,
 * oracle/response.py and oracle/o2.py.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC (no fast-math): the
 * track is evaluated with the same IEEE operations, in the same order, as
 * oracle/track.py, so bin indices, track ends and N_seg agree bit for bit.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>
#include <omp.h>

#define PI 3.141592653589793
#define MSUN_S 4.925490947e-6
#define FDOT_REF 1.34e-12
#define CLIGHT 299792458.0
#define YEAR_S 31557600.0

enum { F_INVALID = 1, F_EMPTY = 2, F_BAND = 4, F_MERGE = 8, F_ALLEXCL = 16 };

typedef struct {
    double M, c8, eta, a2, a3, a4, b2, b3, b4, tc;
} tpl_t;

static void tpl_init(tpl_t *T, double mc, double eta, double f0) {
    double y = 1.0;
    for (int i = 0; i < 12; ++i) {
        double y4 = (y * y) * (y * y);
        y = (4.0 * y + eta / y4) / 5.0;
    }
    T->eta = eta;
    T->M = (mc * MSUN_S) / ((y * y) * y);
    double e2 = eta * eta;
    T->a2 = 743.0 / 2688.0 + (11.0 / 32.0) * eta;
    T->a3 = -3.0 * PI / 10.0;
    T->a4 = (1855099.0 / 14450688.0 + (56975.0 / 258048.0) * eta) + (371.0 / 2048.0) * e2;
    T->b2 = 3715.0 / 8064.0 + (55.0 / 96.0) * eta;
    T->b3 = -3.0 * PI / 4.0;
    T->b4 = (9275495.0 / 14450688.0 + (284875.0 / 258048.0) * eta) + (1855.0 / 2048.0) * e2;
    T->c8 = (8.0 * PI) * T->M;
    double z = T->c8 * f0;
    double r = sqrt(sqrt(z));
    for (int i = 0; i < 10; ++i) r = (2.0 * r + z / (r * r)) / 3.0;
    double th = r;
    for (int i = 0; i < 6; ++i) {
        double th2 = th * th, th3 = th2 * th, th4 = th2 * th2;
        double P = ((1.0 + T->a2 * th2) + T->a3 * th3) + T->a4 * th4;
        double F = th3 * P - z;
        double dP = ((3.0 + (5.0 * T->a2) * th2) + (6.0 * T->a3) * th3) + (7.0 * T->a4) * th4;
        th = th - F / (th2 * dP);
    }
    double th2 = th * th, th4 = th2 * th2, th8 = th4 * th4;
    T->tc = (5.0 * T->M) / (eta * th8);
}

static void tpl_at(const tpl_t *T, double t, double *Phi, double *f, double *fdot, double *A) {
    double tau = T->tc - t;
    double q = (T->eta * tau) / (5.0 * T->M);
    double s = sqrt(sqrt(sqrt(q)));
    double th = 1.0 / s;
    double th2 = th * th, th3 = th2 * th, th4 = th2 * th2;
    double Pf = ((1.0 + T->a2 * th2) + T->a3 * th3) + T->a4 * th4;
    *f = (th3 / T->c8) * Pf;
    double dPf = ((3.0 + (5.0 * T->a2) * th2) + (6.0 * T->a3) * th3) + (7.0 * T->a4) * th4;
    double dfdth = (th2 / T->c8) * dPf;
    double th8 = th4 * th4, th9 = th8 * th;
    double dthdt = (T->eta * th9) / (40.0 * T->M);
    *fdot = dfdth * dthdt;
    double Pp = ((1.0 + T->b2 * th2) + T->b3 * th3) + T->b4 * th4;
    double thm5 = 1.0 / (th4 * th);
    *Phi = -((2.0 * thm5) * Pp) / T->eta;
    *A = pow(*f, 2.0 / 3.0);
}

static int valid_params(double mc, double eta, double f0, double ct, double ci) {
    if (!(mc > 0.0) || !(eta >= 0.01) || !(eta <= 0.25) || !(f0 > 0.0)) return 0;
    if (!(fabs(ct) <= 1.0) || !(fabs(ci) <= 1.0)) return 0;
    if (!isfinite(mc) || !isfinite(eta) || !isfinite(f0) || !isfinite(ct) || !isfinite(ci)) return 0;
    return 1;
}

static int64_t nseg_rule(double fdot0) {
    int n = 0;
    double r2 = sqrt(2.0);
    for (int i = 1; i <= 4; ++i)
        if (fdot0 >= FDOT_REF * ldexp(r2, 3 * i - 2)) ++n;
    return (int64_t)16 << n;
}

/* ---------------------------------------------------------------- Fresnel */
static void fresnel_paper(double z, double *C, double *S) {
    double az = fabs(z);
    double sg = (z > 0.0) ? 1.0 : ((z < 0.0) ? -1.0 : 0.0);
    double arg = (PI / 2.0) * az * az;
    double c = cos(arg), s = sin(arg);
    double Cv, Sv;
    if (az > 6.0) {
        Sv = 0.5 - c / (PI * az);
        Cv = 0.5 + s / (PI * az);
    } else {
        double fz = (1.0 + 0.926 * az) / (2.0 + 1.792 * az + 3.104 * az * az);
        double gz = 1.0 / (2.0 + 4.142 * az + 3.492 * az * az + 6.670 * az * az * az);
        Sv = 0.5 - fz * c - gz * s;
        Cv = 0.5 + fz * s - gz * c;
    }
    *C = Cv * sg;
    *S = Sv * sg;
}

/* ---------------------------------------------------------------- response */
static void orbits(double t, double p[3][3]) {
    double L = 2.5e9 / CLIGHT, R = 1.495978707e11 / CLIGHT;
    double e = L / (2.0 * sqrt(3.0) * R);
    double a = 2.0 * PI * t / YEAR_S;
    for (int i = 0; i < 3; ++i) {
        double b = 2.0 * PI * i / 3.0;
        p[i][0] = R * cos(a) + 0.5 * e * R * (cos(2.0 * a - b) - 3.0 * cos(b));
        p[i][1] = R * sin(a) + 0.5 * e * R * (sin(2.0 * a - b) - 3.0 * sin(b));
        p[i][2] = -sqrt(3.0) * e * R * cos(a - b);
    }
}

typedef struct { double re, im; } cx;
static cx cmul(cx a, cx b) { cx r = {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; return r; }
static cx cadd(cx a, cx b) { cx r = {a.re + b.re, a.im + b.im}; return r; }
static cx csub(cx a, cx b) { cx r = {a.re - b.re, a.im - b.im}; return r; }
static cx cscale(cx a, double s) { cx r = {a.re * s, a.im * s}; return r; }

typedef struct { double k[3], ep[3][3], ex[3][3], ci; } sky_t;

static void sky_init(sky_t *S, double ct, double phi, double psi, double ci) {
    double st = sqrt(1.0 - ct * ct), cp = cos(phi), sp = sin(phi);
    double u[3] = {ct * cp, ct * sp, -st}, v[3] = {sp, -cp, 0.0};
    S->k[0] = -st * cp; S->k[1] = -st * sp; S->k[2] = -ct;
    double c2 = cos(2.0 * psi), s2 = sin(2.0 * psi);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double p0 = u[i] * u[j] - v[i] * v[j];
            double x0 = u[i] * v[j] + v[i] * u[j];
            S->ep[i][j] = c2 * p0 + s2 * x0;
            S->ex[i][j] = -s2 * p0 + c2 * x0;
        }
    S->ci = ci;
}

static double quad3(const double n[3], double e[3][3]) {
    double r = 0.0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) r += n[i] * e[i][j] * n[j];
    return r;
}

/* G_sr for 0-based sender s and receiver r */
static cx link_transfer(const sky_t *S, double p[3][3], int s, int r, double f) {
    double L = 2.5e9 / CLIGHT;
    double d[3], nn = 0.0;
    for (int i = 0; i < 3; ++i) { d[i] = p[r][i] - p[s][i]; nn += d[i] * d[i]; }
    nn = sqrt(nn);
    double n[3] = {d[0] / nn, d[1] / nn, d[2] / nn};
    double kn = n[0] * S->k[0] + n[1] * S->k[1] + n[2] * S->k[2];
    double xp = quad3(n, (double (*)[3])S->ep), xx = quad3(n, (double (*)[3])S->ex);
    cx amp = {(1.0 + S->ci * S->ci) / 2.0 * xp, -S->ci * xx};
    double x = PI * f * L * (1.0 - kn);
    double sinc = (x == 0.0) ? 1.0 : sin(x) / x;
    double kps = 0.0;
    for (int i = 0; i < 3; ++i) kps += (p[s][i] + p[r][i]) * S->k[i];
    double ph = -PI * f * (L + kps);
    cx e = {cos(ph), sin(ph)};
    cx pre = {0.0, -PI * f * L * sinc};
    return cmul(cmul(pre, e), amp);
}

static void transfer_ae(const sky_t *S, double t, double f, cx *TA, cx *TE) {
    double p[3][3];
    orbits(t, p);
    double L = 2.5e9 / CLIGHT;
    cx G[3][3];
    for (int s = 0; s < 3; ++s)
        for (int r = 0; r < 3; ++r)
            if (s != r) G[s][r] = link_transfer(S, p, s, r, f);
    cx D = {cos(-2.0 * PI * f * L), sin(-2.0 * PI * f * L)};
    cx one = {1.0, 0.0};
    cx om = csub(one, cmul(D, D));
#define g(s, r) G[(s) - 1][(r) - 1]
    cx TX = cmul(om, csub(cadd(g(3, 1), cmul(D, g(1, 3))), cadd(g(2, 1), cmul(D, g(1, 2)))));
    cx TY = cmul(om, csub(cadd(g(1, 2), cmul(D, g(2, 1))), cadd(g(3, 2), cmul(D, g(2, 3)))));
    cx TZ = cmul(om, csub(cadd(g(2, 3), cmul(D, g(3, 2))), cadd(g(1, 3), cmul(D, g(3, 1)))));
#undef g
    *TA = cscale(csub(TZ, TX), 1.0 / sqrt(2.0));
    *TE = cscale(cadd(csub(TX, cscale(TY, 2.0)), TZ), 1.0 / sqrt(6.0));
}

/* ---------------------------------------------------------------- layout */
int o2_cpu_layout(int M, int Nt, double dt, int64_t n,
                  const double *mc, const double *eta, const double *f0,
                  const double *ct, const double *ci, int nseg_fixed,
                  int64_t *nseg, int64_t *m_end, int64_t *flags, int nthreads) {
    double dT = (double)M * dt, df = 1.0 / dT, fnyq = 0.5 / dt;
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i) {
        flags[i] = 0; m_end[i] = 0;
        int ok = valid_params(mc[i], eta[i], f0[i], ct[i], ci[i]);
        tpl_t T;
        tpl_init(&T, ok ? mc[i] : 30.0, ok ? eta[i] : 0.25, ok ? f0[i] : 0.01);
        double Phi, f, fd, A;
        tpl_at(&T, 0.0, &Phi, &f, &fd, &A);
        nseg[i] = nseg_fixed > 0 ? nseg_fixed : nseg_rule(fd);
        if (!ok) { flags[i] = F_INVALID; continue; }
        int64_t m = 0;
        for (; m < Nt; ++m) {
            double tm = (double)m * dT;
            if (tm + dT >= T.tc) { flags[i] |= F_MERGE; break; }
            tpl_at(&T, tm, &Phi, &f, &fd, &A);
            if ((f + fd * dT >= fnyq - 11.0 * df) || (fd * dT > 10.0 * df)) { flags[i] |= F_BAND; break; }
        }
        m_end[i] = m;
        if (m == 0) flags[i] |= F_EMPTY;
    }
    return 0;
}

/* ---------------------------------------------------------------- statistic */
/* pix: [C][K][Nt] complex stored as (re, im) pairs, K = M/2 + 1. */
int o2_cpu_statistic(int C, int M, int Nt, double dt,
                     const double *pix, const double *u, const double *w, int64_t n,
                     const double *mc, const double *eta, const double *f0, const double *ct,
                     const double *phi, const double *psi, const double *ci,
                     const int64_t *nseg, const int64_t *seg_offset, const int64_t *m_end,
                     int64_t *flags, double *seg_terms, double *stat, double *seg_zn, int nthreads) {
    const int K = M / 2 + 1;
    const double dT = (double)M * dt;
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < n; ++i) {
        const int64_t ns = nseg[i], off = seg_offset[i];
        for (int64_t s = 0; s < ns; ++s) {
            seg_terms[off + s] = 0.0;
            if (seg_zn) { seg_zn[3 * (off + s)] = 0.0; seg_zn[3 * (off + s) + 1] = 0.0; seg_zn[3 * (off + s) + 2] = 0.0; }
        }
        stat[i] = 0.0;
        if (flags[i] & (F_INVALID | F_EMPTY)) continue;
        tpl_t T;
        tpl_init(&T, mc[i], eta[i], f0[i]);
        sky_t S;
        sky_init(&S, ct[i], phi[i], psi[i], ci[i]);
        double zr = 0.0, zi = 0.0, NN = 0.0, total = 0.0;
        int64_t cur = 0;
        int any = 0;
        for (int64_t m = 0; m <= m_end[i]; ++m) {
            int64_t sg = (m < m_end[i]) ? (m * ns) / Nt : ns;
            while (cur < sg) { /* close segment cur */
                double v = (NN > 0.0) ? 2.0 * (zr * zr + zi * zi) / NN : 0.0;
                seg_terms[off + cur] = v;
                if (seg_zn) { seg_zn[3 * (off + cur)] = zr; seg_zn[3 * (off + cur) + 1] = zi; seg_zn[3 * (off + cur) + 2] = NN; }
                if (NN > 0.0) any = 1;
                total += v;
                zr = zi = NN = 0.0;
                ++cur;
            }
            if (m == m_end[i]) break;
            double wm = w[m];
            if (wm == 0.0) continue;
            double tm = (double)m * dT;
            double Phi, f, fd, A;
            tpl_at(&T, tm, &Phi, &f, &fd, &A);
            double kc = ceil(f * dT);
            cx TC[2];
            transfer_ae(&S, tm, f, &TC[0], &TC[1]);
            double r = sqrt(2.0 * fd);
            for (int j = -10; j <= 10; ++j) {
                int64_t k = (int64_t)kc + j;
                if (k < 1 || k > M / 2 - 1) continue;
                double fk = (double)k / dT;
                double zeta = (f - fk) / fd;
                double v0 = r * zeta, v1 = r * (dT + zeta);
                double C0, S0, C1, S1;
                fresnel_paper(v0, &C0, &S0);
                fresnel_paper(v1, &C1, &S1);
                double dC = C1 - C0, dS = S1 - S0;
                double ph = Phi - PI * fd * zeta * zeta;
                double pref = A / r;
                cx h = {pref * (cos(ph) * dC - sin(ph) * dS), pref * (sin(ph) * dC + cos(ph) * dS)};
                double wt = u[k] * wm;
                for (int c = 0; c < C; ++c) {
                    cx y = cscale(cmul(TC[c], h), wt);
                    const double *dp = pix + 2 * (((int64_t)c * K + k) * Nt + m);
                    /* conj(D) * Y */
                    zr += dp[0] * y.re + dp[1] * y.im;
                    zi += dp[0] * y.im - dp[1] * y.re;
                    NN += y.re * y.re + y.im * y.im;
                }
            }
        }
        while (cur < ns) { seg_terms[off + cur] = 0.0; ++cur; }
        stat[i] = total;
        if (!any) flags[i] |= F_ALLEXCL;
    }
    return 0;
}

/* Track values of one template at times t[nt]: out[4*i..] = (Phi, f, fdot, A); also tc. */
int o2_cpu_track(double mc, double eta, double f0, int64_t nt, const double *t, double *out, double *tc) {
    tpl_t T;
    tpl_init(&T, mc, eta, f0);
    *tc = T.tc;
    for (int64_t i = 0; i < nt; ++i) tpl_at(&T, t[i], out + 4 * i, out + 4 * i + 1, out + 4 * i + 2, out + 4 * i + 3);
    return 0;
}

/* Per-tranche transfer (T_A, T_E) of one template at times t and frequencies f: out[4*i..] = (ReA, ImA, ReE, ImE). */
int o2_cpu_transfer(double ct, double phi, double psi, double ci, int64_t nt, const double *t, const double *f, double *out) {
    sky_t S;
    sky_init(&S, ct, phi, psi, ci);
    for (int64_t i = 0; i < nt; ++i) {
        cx A, E;
        transfer_ae(&S, t[i], f[i], &A, &E);
        out[4 * i] = A.re; out[4 * i + 1] = A.im; out[4 * i + 2] = E.re; out[4 * i + 3] = E.im;
    }
    return 0;
}
