// Statistic kernels: per-template setup (segment layout), per-tranche
// geometry table, and the bank statistic under two schedules.
//
//   THREAD  one thread per template walks its tranches and bins in order;
//           this is the mapping the paper describes for its own GPU code.
//   WAVE    one 64-lane wavefront per template, lane l on tranche m0 + l,
//           so the 21 per-bin gathers of a wave read 64 consecutive tranches
//           of one frequency layer (contiguous in the LAYER_MAJOR store);
//           tranche sums are reduced across lanes per segment; a persistent
//           grid pulls templates from a device counter.
//
// No kernel allocates; all scratch lives in the caller's workspace.
#include "tfsc_stat_common.hpp"

namespace tfsc {

// ------------------------------------------------------------------ layout
__global__ void k_layout_nseg(int64_t n, const double *__restrict__ mc, const double *__restrict__ ln_mc,
                              const double *__restrict__ eta, const double *__restrict__ f0,
                              const double *__restrict__ ct, const double *__restrict__ ci, int nseg_fixed,
                              int32_t *__restrict__ nseg, int64_t *__restrict__ block_sums) {
    __shared__ int64_t sh[256];
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int v = 0;
    if (i < n) {
        const double mci = bank_mc(mc, ln_mc, i);
        bool ok = params_valid(mci, eta[i], f0[i], ct[i], ci[i]);
        Track T;
        track_init(T, ok ? mci : 30.0, ok ? eta[i] : 0.25, ok ? f0[i] : 0.01);
        double Phi, f, fd;
        track_at(T, 0.0, Phi, f, fd);
        v = nseg_fixed > 0 ? nseg_fixed : nseg_rule(fd);
        nseg[i] = v;
    }
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) block_sums[blockIdx.x] = sh[0];
}

// exclusive scan of block sums in place (one block of 1024 threads)
__global__ void k_scan_blocks(int64_t nb, int64_t *__restrict__ block_sums) {
    __shared__ int64_t sh[1024];
    __shared__ int64_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t base = 0; base < nb; base += 1024) {
        int64_t idx = base + threadIdx.x;
        int64_t v = idx < nb ? block_sums[idx] : 0;
        sh[threadIdx.x] = v;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            int64_t t = (int)threadIdx.x >= off ? sh[threadIdx.x - off] : 0;
            __syncthreads();
            sh[threadIdx.x] += t;
            __syncthreads();
        }
        if (idx < nb) block_sums[idx] = carry + sh[threadIdx.x] - v;
        __syncthreads();
        if (threadIdx.x == 1023) carry += sh[1023];
        __syncthreads();
    }
}

__global__ void k_layout_offsets(int64_t n, const int32_t *__restrict__ nseg, const int64_t *__restrict__ block_base,
                                 int64_t *__restrict__ seg_offset) {
    __shared__ int64_t sh[256];
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t v = i < n ? nseg[i] : 0;
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        int64_t t = (int)threadIdx.x >= off ? sh[threadIdx.x - off] : 0;
        __syncthreads();
        sh[threadIdx.x] += t;
        __syncthreads();
    }
    if (i < n) seg_offset[i + 1] = block_base[blockIdx.x] + sh[threadIdx.x];
    if (i == 0) seg_offset[0] = 0;
}

// ------------------------------------------------------------------ processing order
__global__ void k_zero_u32(uint32_t *p, int n);

// Counting sort of the bank by the frequency bin of f0 and, within it, by a class of ln Mc (invalid rows
// last): bucket histogram, exclusive scan, scatter.  Templates adjacent in the order then share rows for
// longer (similar chirps from the same start), so waves that run at the same time reuse each other's
// pixel rows in L2.  Within a bucket the order follows the atomics.
__device__ __forceinline__ int order_bucket(double f0, double mc, double dT, int K, bool ok) {
    if (!ok) return K * kOrderMcClasses;
    const double b = floor(f0 * dT);
    const int kb = b < 0.0 ? 0 : (b > (double)(K - 1) ? K - 1 : (int)b);
    const double c = floor((log(mc) - kOrderLnMcLo) * (kOrderMcClasses / (kOrderLnMcHi - kOrderLnMcLo)));
    const int mcl = c < 0.0 ? 0 : (c > (double)(kOrderMcClasses - 1) ? kOrderMcClasses - 1 : (int)c);
    return kb * kOrderMcClasses + mcl;
}

__global__ void k_order_hist(int64_t n, const double *__restrict__ mc, const double *__restrict__ ln_mc,
                             const double *__restrict__ eta,
                             const double *__restrict__ f0, const double *__restrict__ ct,
                             const double *__restrict__ ci, double dT, int K, uint32_t *__restrict__ count) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const bool ok = params_valid(bank_mc(mc, ln_mc, i), eta[i], f0[i], ct[i], ci[i]);
    atomicAdd(count + order_bucket(f0[i], ok ? bank_mc(mc, ln_mc, i) : 1.0, dT, K, ok), 1u);
}

// Exclusive scan of count[0..nb) into cursor[0..nb) in three passes: each block of 1024 threads scans 1024
// consecutive buckets (coalesced) and writes its total, one block scans the totals (at most 1024 of them), and
// each block adds its offset.
__device__ __forceinline__ uint32_t block_scan_inclusive_1024(uint32_t v, uint32_t *sh) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const uint32_t t = (int)threadIdx.x >= off ? sh[threadIdx.x - off] : 0u;
        __syncthreads();
        sh[threadIdx.x] += t;
        __syncthreads();
    }
    return sh[threadIdx.x];
}

__global__ void k_order_scan_local(int nb, const uint32_t *__restrict__ count, uint32_t *__restrict__ cursor,
                                   uint32_t *__restrict__ block_tot) {
    __shared__ uint32_t sh[1024];
    const int b = blockIdx.x * 1024 + threadIdx.x;
    const uint32_t v = b < nb ? count[b] : 0u;
    const uint32_t inc = block_scan_inclusive_1024(v, sh);
    if (b < nb) cursor[b] = inc - v;
    if (threadIdx.x == 1023) block_tot[blockIdx.x] = inc;
}

__global__ void k_order_scan_top(int nblk, uint32_t *__restrict__ block_tot) {
    __shared__ uint32_t sh[1024];
    const uint32_t v = (int)threadIdx.x < nblk ? block_tot[threadIdx.x] : 0u;
    const uint32_t inc = block_scan_inclusive_1024(v, sh);
    if ((int)threadIdx.x < nblk) block_tot[threadIdx.x] = inc - v;
}

__global__ void k_order_scan_add(int nb, uint32_t *__restrict__ cursor, const uint32_t *__restrict__ block_off) {
    const int b = blockIdx.x * 1024 + threadIdx.x;
    if (b < nb) cursor[b] += block_off[blockIdx.x];
}

__global__ void k_order_scatter(int64_t n, const double *__restrict__ mc, const double *__restrict__ ln_mc,
                             const double *__restrict__ eta,
                                const double *__restrict__ f0, const double *__restrict__ ct,
                                const double *__restrict__ ci, double dT, int K, uint32_t *__restrict__ cursor,
                                int32_t *__restrict__ order) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const bool ok = params_valid(bank_mc(mc, ln_mc, i), eta[i], f0[i], ct[i], ci[i]);
    const uint32_t pos = atomicAdd(cursor + order_bucket(f0[i], ok ? bank_mc(mc, ln_mc, i) : 1.0, dT, K, ok), 1u);
    order[pos] = (int32_t)i;
}

hipError_t launch_order(const OrderLaunch &L, hipStream_t st) {
    if (L.n == 0) return hipSuccess;
    const int K = L.M / 2 + 1, nb = K * kOrderMcClasses + 1;
    const double dT = (double)L.M * L.dt;
    const int nblk = (nb + 1023) / 1024;  // at most 1024: K <= 2049 and 256 classes
    if (nblk > 1024) return hipErrorInvalidValue;
    uint32_t *count = L.ws, *cursor = L.ws + nb, *block_tot = L.ws + 2 * nb;
    const unsigned blocks = (unsigned)((L.n + 255) / 256);
    hipLaunchKernelGGL(k_zero_u32, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, st, count, nb);
    hipLaunchKernelGGL(k_order_hist, dim3(blocks), dim3(256), 0, st, L.n, L.mc, L.ln_mc, L.eta, L.f0, L.ct, L.ci, dT, K,
                       count);
    hipLaunchKernelGGL(k_order_scan_local, dim3((unsigned)nblk), dim3(1024), 0, st, nb, count, cursor, block_tot);
    hipLaunchKernelGGL(k_order_scan_top, dim3(1), dim3(1024), 0, st, nblk, block_tot);
    hipLaunchKernelGGL(k_order_scan_add, dim3((unsigned)nblk), dim3(1024), 0, st, nb, cursor, block_tot);
    hipLaunchKernelGGL(k_order_scatter, dim3(blocks), dim3(256), 0, st, L.n, L.mc, L.ln_mc, L.eta, L.f0, L.ct, L.ci, dT, K,
                       cursor, L.order);
    return hipGetLastError();
}

// ------------------------------------------------------------------ geometry
// Rigid analytic orbits (first order in e = L / (2 sqrt 3 R)): spacecraft positions at time t, light-seconds.
__device__ inline void analytic_positions(double t, double p[3][3]) {
    const double L = kArmM / kClight, R = kAuM / kClight;
    const double e = L / (2.0 * sqrt(3.0) * R);
    double a = kTwoPi * t / kYearS;
    for (int i = 0; i < 3; ++i) {
        double b = kTwoPi * i / 3.0;
        double sa, ca, s2, c2, sb, cb, s1, c1;
        sincos(a, &sa, &ca);
        sincos(2.0 * a - b, &s2, &c2);
        sincos(b, &sb, &cb);
        sincos(a - b, &s1, &c1);
        p[i][0] = R * ca + 0.5 * e * R * (c2 - 3.0 * cb);
        p[i][1] = R * sa + 0.5 * e * R * (s2 - 3.0 * sb);
        p[i][2] = -sqrt(3.0) * e * R * c1;
    }
}

// Geometry table of tranche m from the three positions: rows 0..8 the positions, rows 9..17 the unit arm
// vectors n_01, n_12, n_20 (FP64, and their FP32 copy).
__device__ inline void store_geometry(const double p[3][3], int m, int Nt, double *__restrict__ geo,
                                      float *__restrict__ geo32) {
    for (int i = 0; i < 3; ++i)
        for (int x = 0; x < 3; ++x) geo[(size_t)(3 * i + x) * Nt + m] = p[i][x];
    for (int a2 = 0; a2 < 3; ++a2) {
        int s = a2, r = (a2 + 1) % 3;
        double d[3], nn = 0.0;
        for (int x = 0; x < 3; ++x) {
            d[x] = p[r][x] - p[s][x];
            nn += d[x] * d[x];
        }
        nn = sqrt(nn);
        for (int x = 0; x < 3; ++x) {
            geo[(size_t)(9 + 3 * a2 + x) * Nt + m] = d[x] / nn;
            geo32[(size_t)(3 * a2 + x) * Nt + m] = (float)(d[x] / nn);
        }
    }
}

// The analytic orbit at t_m = m dT.
__global__ void k_geometry(int Nt, double dT, double *__restrict__ geo, float *__restrict__ geo32) {
    int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= Nt) return;
    double p[3][3];
    analytic_positions((double)m * dT, p);
    store_geometry(p, m, Nt, geo, geo32);
}

// A caller's orbit: positions orbit[(3 i + x) Nt + m] of spacecraft i, coordinate x at t_m (light-seconds),
// e.g. a numerical orbit; the arm vectors are formed from them as for the analytic orbit.
__global__ void k_geometry_table(int Nt, const double *__restrict__ orbit, double *__restrict__ geo,
                                 float *__restrict__ geo32) {
    int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= Nt) return;
    double p[3][3];
    for (int i = 0; i < 3; ++i)
        for (int x = 0; x < 3; ++x) p[i][x] = orbit[(size_t)(3 * i + x) * Nt + m];
    store_geometry(p, m, Nt, geo, geo32);
}

// The analytic orbit's positions in the caller's table layout [3 spacecraft][3 coordinates][Nt].
__global__ void k_orbit_positions(int Nt, double dT, double *__restrict__ out) {
    int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= Nt) return;
    double p[3][3];
    analytic_positions((double)m * dT, p);
    for (int i = 0; i < 3; ++i)
        for (int x = 0; x < 3; ++x) out[(size_t)(3 * i + x) * Nt + m] = p[i][x];
}

// Link light times without point-ahead: out[l Nt + m] = |p_r - p_s| of link row l (rows 0..2: s = a -> r = a + 1 of arm a; rows 3..5 the reverse
// links) at tranche m, from the caller's positions orbit[(3 i + x) Nt + m] or the analytic orbit.
__global__ void k_link_lengths(int Nt, double dT, const double *__restrict__ orbit, double *__restrict__ out) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= Nt) return;
    double p[3][3];
    if (orbit) {
        for (int i = 0; i < 3; ++i)
            for (int x = 0; x < 3; ++x) p[i][x] = orbit[(size_t)(3 * i + x) * Nt + m];
    } else {
        analytic_positions((double)m * dT, p);
    }
    for (int a = 0; a < 3; ++a) {
        const int s = a, r = (a + 1) % 3;
        const double dx = p[r][0] - p[s][0], dy = p[r][1] - p[s][1], dz = p[r][2] - p[s][2];
        const double len = sqrt(dx * dx + dy * dy + dz * dz);
        out[(size_t)a * Nt + m] = len;
        out[(size_t)(3 + a) * Nt + m] = len;
    }
}

hipError_t launch_link_lengths(int Nt, double dT, const double *orbit, double *out, hipStream_t st) {
    hipLaunchKernelGGL(k_link_lengths, dim3((Nt + 127) / 128), dim3(128), 0, st, Nt, dT, orbit, out);
    return hipGetLastError();
}

// Exact power-of-two normalisation of the template weights: scale = 2^-e with e the
// binary exponent of max_k u_k, so that max_k u_k * scale lies in [1/2, 1).  Upsilon is
// invariant to it; it keeps |h u|^2 inside the FP32 range (u_k ~ 1e20 in strain units).
__global__ void k_weight_scale(int K, const double *__restrict__ inv_asd, double *__restrict__ scale_out) {
    __shared__ double sh[256];
    // bins 1 .. K - 2 only: DC and Nyquist never enter the statistic
    double v = 0.0;
    for (int k = 1 + threadIdx.x; k < K - 1; k += blockDim.x) {
        double u = inv_asd[k];
        if (isfinite(u) && u > v) v = u;
    }
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + o]);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        int e = 0;
        double mx = sh[0];
        if (mx > 0.0) frexp(mx, &e);
        scale_out[0] = ldexp(1.0, -e);
    }
}

__global__ void k_zero_u32(uint32_t *p, int n) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

// ------------------------------------------------------------------ statistic kernels (bodies in tfsc_stat_common.hpp)
template <int C, class R, class PixT, int LAYOUT, bool RHO>
__global__ __launch_bounds__(256) void k_stat_thread(StatArgs a) {
    stat_thread_body<C, R, PixT, LAYOUT, RHO, kFresnelPaper>(a);
}

template <int C, class R, class PixT, int LAYOUT, bool RHO>
__global__ __launch_bounds__(256, 4) void k_stat_wave(StatArgs a) {
    stat_wave_body<C, R, PixT, LAYOUT, RHO, kFresnelPaper>(a);
}

// ------------------------------------------------------------------ WAVE schedule, several realisations
// The same statistic for RR noise realisations of one grid in one pass over the bank (a design
// alternative for the batching workload: one template's track, spectrum and response serve
// every realisation of the group).  Per tranche the 21 weighted template bins c_j (exact form
// on the wave's band, asymptotic form elsewhere) and Q = sum |c_j|^2 are formed once and parked
// in LDS; each realisation then only gathers its pixels and forms P_c = sum_j conj(D_cj) c_j.
// The segment state of realisation r (its z_n and running Upsilon) lives in lane r, the norm
// N_n is shared.
template <class R>
__device__ __forceinline__ void wave_tranche_coefs(const TrancheSpec<R> &ts, int kc, const R *__restrict__ u_pad,
                                                   int jA, int jB, cx<R> *cf, int lane, R &Q) {
#pragma clang fp contract(fast)
    const R *uk = u_pad + kc;  // uk[jj] = u_{kc + jj - 10}
    Q = (R)0;
#pragma unroll
    for (int jj = 0; jj < 2 * kHalfBins + 1; ++jj) {
        const int j = jj - kHalfBins;
        const R xj = ts.x - (R)j;
        const R w = uk[jj];
        cx<R> g;
        if (j >= jA && j <= jB) {
            const cx<R> h = bin_full(ts, xj, j);
            g = {h.re * w, h.im * w};
        } else {
            g = bin_fast_weighted(ts, xj, w);
        }
        Q += g.re * g.re;
        Q += g.im * g.im;
        cf[jj * 64 + lane] = g;
    }
}

// Per-pixel PSD factor on a lane's coefficient table (the same for every realisation): c_j *= rho at
// (bin kc + j, tranche m), Q recomputed in the same order; rows below 0 already have weight 0.  A
// separate pass, taken only when rho is set, so the table's own loop keeps its registers.
template <class R>
__device__ __forceinline__ void wave_tranche_coefs_rho(cx<R> *cf, int lane, int kc, int m, int Nt,
                                                       const float *__restrict__ rho, R &Q) {
#pragma clang fp contract(fast)
    Q = (R)0;
#pragma unroll 1
    for (int jj = 0; jj < 2 * kHalfBins + 1; ++jj) {
        const R r = (R)rho[max(kc + jj - kHalfBins, 0) * Nt + m];  // K Nt < 2^31 (the store is < 4 GiB)
        cx<R> g = cf[jj * 64 + lane];
        g.re *= r;
        g.im *= r;
        cf[jj * 64 + lane] = g;
        Q += g.re * g.re;
        Q += g.im * g.im;
    }
}

// P_c = sum_j conj(D_cj) c_j for one realisation (soff0 = its byte offset in the block);
// loads in groups of three, issued before the group's arithmetic.  low: some lane of the
// wave has kc < 10, so rows are per lane and clamped at 0 (their weight is 0).
template <int C, class R, class PixT, int LAYOUT>
__device__ __forceinline__ void wave_tranche_mac(const cx<R> *cf, int lane, int kc, int m, int Nt, int K,
                                                 __amdgpu_buffer_rsrc_t rsrc, uint32_t soff0, bool low, cx<R> (&P)[C]) {
#pragma clang fp contract(fast)
    constexpr uint32_t B = sizeof(PixT) == 8 ? 16u : 8u;
    constexpr uint32_t BP = LAYOUT == 2 ? (uint32_t)C * B : B;
    constexpr int NB = 2 * kHalfBins + 1, G = 3;
    const uint32_t row = (uint32_t)Nt * BP, chan = (uint32_t)K * row;
    const uint32_t voff = (uint32_t)((kc - kHalfBins) * Nt + m) * BP;
#pragma unroll
    for (int c = 0; c < C; ++c) P[c] = {(R)0, (R)0};
#pragma unroll
    for (int j0 = 0; j0 < NB; j0 += G) {
        cx<typename PixTraits<PixT>::R> Dl[G][C];
#pragma unroll
        for (int u = 0; u < G; ++u) {
            // low: the lane's own row, clamped at 0 (a per-lane offset; no branch per bin)
            const int k = max(kc - kHalfBins + j0 + u, 0);
            const uint32_t v = low ? (uint32_t)(k * Nt + m) * BP : voff;
            const uint32_t so = low ? soff0 : soff0 + (uint32_t)(j0 + u) * row;
            bin_pixels<C, PixT, LAYOUT>(rsrc, v, so, chan, Dl[u]);
        }
#pragma unroll
        for (int u = 0; u < G; ++u) {
            const cx<R> g = cf[(j0 + u) * 64 + lane];
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const R dr = (R)Dl[u][c].re, di = (R)Dl[u][c].im;
                P[c].re += dr * g.re;
                P[c].re += di * g.im;
                P[c].im += dr * g.im;
                P[c].im -= di * g.re;
            }
        }
    }
}

// Segment state of the multi-realisation kernel: N, cur and any are wave-uniform; zr, zi and
// total belong to the realisation of the lane (lanes >= RR carry zeros).
struct SegAccMulti {
    double zr, zi, total;  // per lane
    double N;              // shared
    int cur;
    bool any;
};

__device__ __forceinline__ void close_segments_multi(SegAccMulti &acc, int upto, int64_t off, double *seg_terms,
                                                     int64_t seg_stride, bool owner, int lane) {
    while (acc.cur < upto) {
        const double v = acc.N > 0.0 ? 2.0 * (acc.zr * acc.zr + acc.zi * acc.zi) / acc.N : 0.0;
        // a plane shorter than the segment layout (a caller error) loses terms instead of overrunning
        if (owner && off + acc.cur < seg_stride) seg_terms[(int64_t)lane * seg_stride + off + acc.cur] = v;
        if (acc.N > 0.0) acc.any = true;
        acc.total += v;
        acc.zr = acc.zi = acc.N = 0.0;
        ++acc.cur;
    }
}

template <int C, class R, class PixT, int LAYOUT, int RR>
__global__ __launch_bounds__(256, 4) void k_stat_wave_multi(StatArgs a) {
    // LDS: u_pad[K + 20] (weights, as in k_stat_wave), then per wave the 21 weighted template
    // bins of each lane's tranche, cf[j][lane], and the tranche sums of its RR realisations,
    // zbuf[r][lane] = (Re z, Im z).
    extern __shared__ unsigned char smem_raw[];
    const int KP = a.K + 2 * kHalfBins;
    R *u_pad = reinterpret_cast<R *>(smem_raw);
    const size_t zoff = ((sizeof(R) * (size_t)KP + 15) / 16) * 16;
    cx<R> *cfbuf = reinterpret_cast<cx<R> *>(smem_raw + zoff) + (size_t)(threadIdx.x >> 6) * (2 * kHalfBins + 1 + RR) * 64;
    cx<R> *zbuf = cfbuf + (2 * kHalfBins + 1) * 64;
    const double u_mul = a.u_scale[0];
    const int kmax = a.M / 2 - 1;
    for (int q = threadIdx.x; q < KP; q += blockDim.x) {
        const int k = q - kHalfBins;
        u_pad[q] = (k >= 1 && k <= kmax) ? (R)(a.inv_asd[k] * u_mul) : (R)0;
    }
    __syncthreads();
    const __amdgpu_buffer_rsrc_t rsrc = pix_rsrc(a.pix, a.pix_bytes);
    const GeoView gv = geo_view(a.geo, a.geo32, a.Nt);
    double *const seg_terms = a.seg_terms + (int64_t)a.rho0 * a.seg_stride;
    double *const stat = a.stat + (int64_t)a.rho0 * a.n;

    const int lane = threadIdx.x & 63;
    const bool owner = lane < RR;  // lane r holds realisation rho0 + r
    for (;;) {
        const uint32_t mine = atomicAdd(a.counter, lane == 0 ? 1u : 0u);
        const int64_t item = (int64_t)__builtin_amdgcn_readfirstlane(mine);
        if (item >= a.n) break;
        const int64_t i = a.order ? (int64_t)__builtin_amdgcn_readfirstlane(a.order[item]) : item;
        if (i < 0 || i >= a.n) continue;  // malformed processing order: skip rather than fault
        const int ns = a.nseg[i];
        const int64_t off = a.seg_offset[i];
        SegAccMulti acc{0, 0, 0, 0, 0, false};
        int flag = 0;
        if (!params_valid(a.mc[i], a.eta[i], a.f0[i], a.ct[i], a.ci[i])) {
            close_segments_multi(acc, ns, off, seg_terms, a.seg_stride, owner, lane);
            if (owner) stat[(int64_t)lane * a.n + i] = 0.0;
            if (lane == 0 && a.rho0 == 0) {
                a.flags[i] = kFlagInvalid;
                if (a.n_active) a.n_active[i] = 0;
            }
            continue;
        }
        Track T;
        track_init(T, a.mc[i], a.eta[i], a.f0[i]);
        wave_uniform(T);
        Sky<R> S;
        sky_init(S, a.ct[i], a.phi[i], a.psi[i], a.ci[i]);
        wave_uniform(S);
        int m_end = a.Nt, n_act = 0;
        SegWalk sw;
        sw.init(a.Nt, ns);
        for (int m0 = 0; m0 < m_end; m0 += 64) {
            const int m = m0 + lane;
            const bool inr = m < a.Nt;
            const double wm_raw = inr ? a.tranche_w[m] : 0.0;
            double Phi, f, fdot;
            int code = track_step_lanes(T, (double)(inr ? m : a.Nt - 1) * a.dT, a.dT, a.df, a.fnyq, Phi, f, fdot);
            code = inr ? code : 0;
            const uint64_t viol = __ballot(code != 0);
            int lim = a.Nt;
            if (viol) {
                const int first = __builtin_amdgcn_readfirstlane(__ffsll((unsigned long long)viol) - 1);
                lim = m0 + first;
                flag |= __builtin_amdgcn_readlane(code, first);
                m_end = lim;
            }
            const bool active = inr && m < lim;
            const double wmd = active ? wm_raw : 0.0;
            const bool work = active && wmd != 0.0;
            n_act += __popcll(__ballot(work));
            TrancheSpec<R> ts;
            int kc = 0;
            int nlo = INT_MIN, hi = INT_MIN;
            if (work) {
                kc = tranche_setup(ts, Phi, f, fdot, a.dT);
                nlo = -ts.j0lo;
                hi = ts.j1hi;
            }
            wave_max2_i32(nlo, hi);
            const int jA = -nlo;
            const int jB = hi;
            const bool low = __ballot(work && kc < kHalfBins) != 0;
            R nn = 0;
            if (work) {
                // the response first, so its temporaries are gone before the bins are formed
                cx<R> TA, TE;
                transfer_ae(S, gv, m, f, TA, TE);
                R tt = TA.re * TA.re + TA.im * TA.im;
                if constexpr (C == 2) tt += TE.re * TE.re + TE.im * TE.im;
                R Q;
                wave_tranche_coefs<R>(ts, kc, u_pad, jA, jB, cfbuf, lane, Q);
                if (a.rho) wave_tranche_coefs_rho<R>(cfbuf, lane, kc, m, a.Nt, a.rho, Q);
                const R wm = (R)wmd;
                nn = wm * wm * tt * Q;
#pragma unroll 1
                for (int r = 0; r < RR; ++r) {
                    cx<R> P[C];
                    wave_tranche_mac<C, R, PixT, LAYOUT>(cfbuf, lane, kc, m, a.Nt, a.K, rsrc,
                                                         (uint32_t)(a.rho0 + r) * a.real_stride, low, P);
                    cx<R> z = cmul(TA, P[0]);
                    if constexpr (C == 2) z = cadd(z, cmul(TE, P[1]));
                    zbuf[r * 64 + lane] = {wm * z.re, wm * z.im};
                }
            } else {
#pragma unroll 1
                for (int r = 0; r < RR; ++r) zbuf[r * 64 + lane] = {(R)0, (R)0};
            }
            const int last = min(min(m0 + 63, lim - 1), a.Nt - 1);
            if (last >= m0) {
                while (sw.hi <= m0) sw.step();
                for (;;) {
                    const bool in_seg = active && m >= sw.lo && m < sw.hi;
                    R vn = in_seg ? nn : (R)0;
                    vn = wave_sum<R>(vn);
                    close_segments_multi(acc, sw.s, off, seg_terms, a.seg_stride, owner, lane);
                    acc.N += (double)vn;
                    // realisation sums: lane r keeps realisation r's
                    double myr = 0.0, myi = 0.0;
#pragma unroll 1
                    for (int r = 0; r < RR; r += 2) {
                        const cx<R> z0 = zbuf[r * 64 + lane];
                        const cx<R> z1 = r + 1 < RR ? zbuf[(r + 1) * 64 + lane] : cx<R>{(R)0, (R)0};
                        R v0 = in_seg ? z0.re : (R)0, v1 = in_seg ? z0.im : (R)0, v2 = in_seg ? z1.re : (R)0;
                        wave_sum3<R>(v0, v1, v2);
                        R v3 = in_seg ? z1.im : (R)0;
                        v3 = wave_sum<R>(v3);
                        myr = lane == r ? (double)v0 : (lane == r + 1 ? (double)v2 : myr);
                        myi = lane == r ? (double)v1 : (lane == r + 1 ? (double)v3 : myi);
                    }
                    acc.zr += myr;
                    acc.zi += myi;
                    if (sw.hi > last) break;
                    sw.step();
                }
            }
            if (viol) break;
        }
        if (m_end == 0) flag |= kFlagEmpty;
        close_segments_multi(acc, ns, off, seg_terms, a.seg_stride, owner, lane);
        if (!acc.any && m_end > 0) flag |= kFlagAllExcluded;
        if (owner) stat[(int64_t)lane * a.n + i] = acc.total;
        if (lane == 0 && a.rho0 == 0) {
            a.flags[i] = flag;
            if (a.n_active) a.n_active[i] = n_act;
        }
    }
}

// ------------------------------------------------------------------ track inspection
__global__ void k_track(int64_t n, int Nt, double dt, double dT, const double *__restrict__ mc,
                        const double *__restrict__ ln_mc, const double *__restrict__ eta,
                        const double *__restrict__ f0, const double *__restrict__ ct, const double *__restrict__ ci,
                        double *__restrict__ out) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * Nt) return;
    int64_t i = e / Nt;
    int m = (int)(e % Nt);
    double *o = out + 4 * e;
    o[0] = o[1] = o[2] = 0.0;
    const double mci = bank_mc(mc, ln_mc, i);
    if (!params_valid(mci, eta[i], f0[i], ct[i], ci[i])) {
        o[3] = (double)kFlagInvalid;
        return;
    }
    Track T;
    track_init(T, mci, eta[i], f0[i]);
    double Phi = 0.0, f = 0.0, fdot = 0.0;
    int code = track_step(T, (double)m * dT, dT, 1.0 / dT, 0.5 / dt, Phi, f, fdot);
    if (code != kFlagMergeEnd) {
        o[0] = Phi;
        o[1] = f;
        o[2] = fdot;
    }
    o[3] = (double)code;
}

hipError_t launch_track(int64_t n, int M, int Nt, double dt, const double *mc, const double *ln_mc, const double *eta,
                        const double *f0, const double *ct, const double *ci, double *out, hipStream_t st) {
    int64_t tot = n * (int64_t)Nt;
    if (tot == 0) return hipSuccess;
    hipLaunchKernelGGL(k_track, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, n, Nt, dt, (double)M * dt, mc,
                       ln_mc, eta, f0, ct, ci, out);
    return hipGetLastError();
}

// ------------------------------------------------------------------ launchers
hipError_t launch_layout(const LayoutLaunch &L, hipStream_t st) {
    int64_t nb = (L.n + 255) / 256;
    if (L.n == 0) {
        hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, st, reinterpret_cast<uint32_t *>(L.seg_offset), 2);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_layout_nseg, dim3((unsigned)nb), dim3(256), 0, st, L.n, L.mc, L.ln_mc, L.eta, L.f0, L.ct,
                       L.ci, L.nseg_fixed, L.nseg, L.block_sums);
    hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(1024), 0, st, nb, L.block_sums);
    hipLaunchKernelGGL(k_layout_offsets, dim3((unsigned)nb), dim3(256), 0, st, L.n, L.nseg, L.block_sums,
                       L.seg_offset);
    return hipGetLastError();
}

hipError_t launch_geometry(int Nt, double dT, const double *orbit, double *geo, hipStream_t st) {
    if (orbit)
        hipLaunchKernelGGL(k_geometry_table, dim3((Nt + 127) / 128), dim3(128), 0, st, Nt, orbit, geo,
                           geo32_of(geo, Nt));
    else
        hipLaunchKernelGGL(k_geometry, dim3((Nt + 127) / 128), dim3(128), 0, st, Nt, dT, geo, geo32_of(geo, Nt));
    return hipGetLastError();
}

hipError_t launch_orbit_positions(int Nt, double dT, double *out, hipStream_t st) {
    hipLaunchKernelGGL(k_orbit_positions, dim3((Nt + 127) / 128), dim3(128), 0, st, Nt, dT, out);
    return hipGetLastError();
}


template <int C, class R, class PixT>
static hipError_t launch_thread_t(const StatArgs &a, int layout, hipStream_t st) {
    dim3 grid((unsigned)((a.n + 255) / 256)), block(256);
    if (a.rho) {
        if (layout == 0)
            hipLaunchKernelGGL((k_stat_thread<C, R, PixT, 0, true>), grid, block, 0, st, a);
        else if (layout == 1)
            hipLaunchKernelGGL((k_stat_thread<C, R, PixT, 1, true>), grid, block, 0, st, a);
        else
            hipLaunchKernelGGL((k_stat_thread<C, R, PixT, 2, true>), grid, block, 0, st, a);
        return hipGetLastError();
    }
    if (layout == 0)
        hipLaunchKernelGGL((k_stat_thread<C, R, PixT, 0, false>), grid, block, 0, st, a);
    else if (layout == 1)
        hipLaunchKernelGGL((k_stat_thread<C, R, PixT, 1, false>), grid, block, 0, st, a);
    else
        hipLaunchKernelGGL((k_stat_thread<C, R, PixT, 2, false>), grid, block, 0, st, a);
    return hipGetLastError();
}

template <int C, class R, class PixT>
static hipError_t launch_wave_t(const StatArgs &a, int layout, int n_groups, int block_waves, hipStream_t st) {
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, st, a.counter, 1);
    const size_t KP = (size_t)a.K + 2 * kHalfBins;
    size_t shmem = sizeof(R) * KP + (PixTraits<PixT>::scaled ? sizeof(float) * C * KP : 0);
    if constexpr (!PixTraits<PixT>::scaled) {
        if (a.rho) {
            if (layout == 2)
                hipLaunchKernelGGL((k_stat_wave<C, R, PixT, 2, true>), dim3(n_groups), dim3(64 * block_waves), shmem,
                                   st, a);
            else
                hipLaunchKernelGGL((k_stat_wave<C, R, PixT, 0, true>), dim3(n_groups), dim3(64 * block_waves), shmem,
                                   st, a);
            return hipGetLastError();
        }
    } else {
        if (a.rho) return hipErrorInvalidValue;
    }
    if (layout == 2)
        hipLaunchKernelGGL((k_stat_wave<C, R, PixT, 2, false>), dim3(n_groups), dim3(64 * block_waves), shmem, st, a);
    else
        hipLaunchKernelGGL((k_stat_wave<C, R, PixT, 0, false>), dim3(n_groups), dim3(64 * block_waves), shmem, st, a);
    return hipGetLastError();
}

template <int C, class R>
static hipError_t dispatch_pix(const StatLaunch &L, const StatArgs &a, hipStream_t st) {
    switch (L.pix_dtype) {
        case 0:
            if constexpr (sizeof(R) == 8) {
                return L.schedule == 0 ? launch_thread_t<C, R, double>(a, L.layout, st)
                                       : launch_wave_t<C, R, double>(a, L.layout, L.n_groups, L.block_waves, st);
            } else {
                return hipErrorInvalidValue;
            }
        case 1:
            return L.schedule == 0 ? launch_thread_t<C, R, float>(a, L.layout, st)
                                   : launch_wave_t<C, R, float>(a, L.layout, L.n_groups, L.block_waves, st);
        case 2:
            if constexpr (sizeof(R) == 4)
                return L.schedule == 0 ? launch_thread_t<C, R, __hip_bfloat16>(a, L.layout, st)
                                       : launch_wave_t<C, R, __hip_bfloat16>(a, L.layout, L.n_groups, L.block_waves, st);
            else
                return hipErrorInvalidValue;
        case 3:
            if constexpr (sizeof(R) == 4)
                return L.schedule == 0 ? launch_thread_t<C, R, __half>(a, L.layout, st)
                                       : launch_wave_t<C, R, __half>(a, L.layout, L.n_groups, L.block_waves, st);
            else
                return hipErrorInvalidValue;
        case 4:
            if constexpr (sizeof(R) == 4)
                return L.schedule == 0 ? launch_thread_t<C, R, int16_t>(a, L.layout, st)
                                       : launch_wave_t<C, R, int16_t>(a, L.layout, L.n_groups, L.block_waves, st);
            else
                return hipErrorInvalidValue;
    }
    return hipErrorInvalidValue;
}

// Chirp masses of a bank given in ln Mc, formed once per call for the statistic and VJP kernels.
__global__ void k_exp_mc(int64_t n, const double *__restrict__ ln_mc, double *__restrict__ mc) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) mc[i] = exp(ln_mc[i]);
}

hipError_t launch_exp_mc(int64_t n, const double *ln_mc, double *mc, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_exp_mc, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, ln_mc, mc);
    return hipGetLastError();
}

hipError_t launch_weight_scale(int K, const double *inv_asd, double *scale_out, hipStream_t st) {
    hipLaunchKernelGGL(k_weight_scale, dim3(1), dim3(256), 0, st, K, inv_asd, scale_out);
    return hipGetLastError();
}

template <int C, class R, int RR>
static hipError_t launch_multi_rr(const StatArgs &a, int layout, int n_groups, int block_waves, hipStream_t st) {
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, st, a.counter, 1);
    const size_t KP = (size_t)a.K + 2 * kHalfBins;
    const size_t shmem =
        ((sizeof(R) * KP + 15) / 16) * 16 + (size_t)block_waves * (2 * kHalfBins + 1 + RR) * 64 * sizeof(cx<R>);
    if (shmem > 160 * 1024) return hipErrorInvalidValue;
    static bool attr_set = false;  // the FP64 tables of four waves exceed the 64 KiB default
    if (!attr_set) {
        (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_stat_wave_multi<C, R, R, 2, RR>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_stat_wave_multi<C, R, R, 0, RR>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        attr_set = true;
    }
    if (layout == 2)
        hipLaunchKernelGGL((k_stat_wave_multi<C, R, R, 2, RR>), dim3(n_groups), dim3(64 * block_waves), shmem, st, a);
    else
        hipLaunchKernelGGL((k_stat_wave_multi<C, R, R, 0, RR>), dim3(n_groups), dim3(64 * block_waves), shmem, st, a);
    return hipGetLastError();
}

// Realisations in launches of `group` (each forms the template work once for its group),
// then the remainder in the largest smaller groups.
template <int C, class R>
static hipError_t launch_multi_t(const StatLaunch &L, StatArgs a, hipStream_t st) {
    for (int r0 = 0; r0 < L.n_real;) {
        a.rho0 = r0;
        const int left = L.n_real - r0;
        int g = L.multi_group;
        while (g > left) g >>= 1;
        hipError_t e;
        switch (g) {
            case 8: e = launch_multi_rr<C, R, 8>(a, L.layout, L.n_groups, L.block_waves, st); break;
            case 4: e = launch_multi_rr<C, R, 4>(a, L.layout, L.n_groups, L.block_waves, st); break;
            case 2: e = launch_multi_rr<C, R, 2>(a, L.layout, L.n_groups, L.block_waves, st); break;
            default: e = launch_multi_rr<C, R, 1>(a, L.layout, L.n_groups, L.block_waves, st); g = 1; break;
        }
        if (e != hipSuccess) return e;
        r0 += g;
    }
    return hipSuccess;
}

hipError_t launch_statistic_multi(const StatLaunch &L, hipStream_t st) {
    StatArgs a = make_args(L);
    if (L.n == 0 || L.n_real == 0) return hipSuccess;
    const uint64_t tot = (uint64_t)L.real_stride * (uint64_t)L.n_real;
    a.pix_bytes = tot > 0xffffffffull ? 0xffffffffu : (uint32_t)tot;
    a.real_stride = (uint32_t)L.real_stride;
    a.seg_stride = L.seg_stride;
    if (L.precision == 0) {
        if (L.pix_dtype != 0) return hipErrorInvalidValue;
        return L.C == 1 ? launch_multi_t<1, double>(L, a, st) : launch_multi_t<2, double>(L, a, st);
    }
    if (L.pix_dtype != 1) return hipErrorInvalidValue;
    if (L.C == 3) return hipErrorInvalidValue;
    return L.C == 1 ? launch_multi_t<1, float>(L, a, st) : launch_multi_t<2, float>(L, a, st);
}

hipError_t launch_statistic(const StatLaunch &L, hipStream_t st) {
    StatArgs a = make_args(L);
    if (L.n == 0) return hipSuccess;
    if (L.C == 1) return L.precision == 0 ? dispatch_pix<1, double>(L, a, st) : dispatch_pix<1, float>(L, a, st);
    if (L.C == 3) return L.precision == 0 ? dispatch_pix<3, double>(L, a, st) : dispatch_pix<3, float>(L, a, st);
    return L.precision == 0 ? dispatch_pix<2, double>(L, a, st) : dispatch_pix<2, float>(L, a, st);
}

}  // namespace tfsc
