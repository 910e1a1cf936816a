// Data -> whitened TF pixels (paper Sec. "Implementation details": every
// tranche is Tukey-windowed and Fourier transformed once; per-tranche PSD;
// tranches overlapping gaps are excluded).
//
// One block handles TB consecutive tranches of one channel: each pair of
// tranches is windowed into LDS as the real and imaginary parts of one complex
// sequence, transformed by a radix-2 Stockham FFT (natural order in and out,
// twiddles from a per-block LDS table), split into the two tranches' spectra,
// whitened, and parked in an
// LDS tile [K][TB]; the tile is then written so that the TB tranches of a
// frequency layer are contiguous (LAYER_MAJOR, or LAYER_MAJOR_CI with the channels of a
// pixel adjacent) or the K bins of a tranche are contiguous (TRANCHE_MAJOR).  16-bit stores go through an FP32 staging
// buffer and a second pass that applies a per-layer scale.
#include "tfsc_device.hpp"
#include "tfsc_kernels.hpp"

namespace tfsc {

__device__ __forceinline__ bool psd_ok(double S) { return S > 0.0 && S < __builtin_huge_val(); }

template <class R>
__device__ __forceinline__ R tukey_w(int n, int M, double alpha) {
    if (alpha <= 0.0) return (R)1;
    int nn = min(n, M - 1 - n);
    double width = floor(alpha * (M - 1) / 2.0);
    if ((double)nn > width) return (R)1;
    return (R)(0.5 * (1.0 + cospi(-1.0 + 2.0 * nn / (alpha * (M - 1)))));
}

template <class R>
__device__ __forceinline__ cx<R> twiddle(double frac);  // exp(-2 pi i frac)
template <>
__device__ __forceinline__ cx<double> twiddle<double>(double frac) {
    double s, c;
    sincospi(-2.0 * frac, &s, &c);
    return {c, s};
}
template <>
__device__ __forceinline__ cx<float> twiddle<float>(double frac) {
    float s, c;
    sincospif((float)(-2.0 * frac), &s, &c);
    return {c, s};
}

template <class R, class XT, class OutT, int TB>
__global__ __launch_bounds__(256) void k_transform(TransformLaunch L, double w2) {
    extern __shared__ unsigned char smem_raw[];
    const int M = L.M, K = M / 2 + 1, Nt = L.Nt;
    cx<R> *bufA = reinterpret_cast<cx<R> *>(smem_raw);
    cx<R> *bufB = bufA + M;
    cx<R> *tw = bufB + M;                       // M/2 twiddles exp(-2 pi i k / M)
    cx<R> *tile = tw + M / 2;                   // [K][TB]
    R *win = reinterpret_cast<R *>(tile + (size_t)K * TB);

    const int c = blockIdx.y;
    const int m0 = blockIdx.x * TB;
    for (int k = threadIdx.x; k < M / 2; k += blockDim.x) tw[k] = twiddle<R>((double)k / M);
    for (int n = threadIdx.x; n < M; n += blockDim.x) win[n] = tukey_w<R>(n, M, L.alpha);
    const XT *x = reinterpret_cast<const XT *>(L.x) + (size_t)c * M * Nt;
    __syncthreads();

    // Two real tranches per complex FFT: z = x_m + i x_{m+1}, whose transform Z gives
    // X_m[k] = (Z[k] + conj Z[M-k]) / 2 and X_{m+1}[k] = (Z[k] - conj Z[M-k]) / (2i).
    static_assert(TB % 2 == 0, "tranches are transformed in pairs");
    for (int tt = 0; tt < TB; tt += 2) {
        const int m = m0 + tt;
        if (m >= Nt) break;  // uniform across the block
        const bool two = m + 1 < Nt;
        for (int n = threadIdx.x; n < M; n += blockDim.x)
            bufA[n] = {(R)x[(size_t)m * M + n] * win[n], two ? (R)x[(size_t)(m + 1) * M + n] * win[n] : (R)0};
        __syncthreads();
        cx<R> *src = bufA, *dst = bufB;
        for (int Ns = 1; Ns < M; Ns <<= 1) {
            for (int j = threadIdx.x; j < M / 2; j += blockDim.x) {
                const int kk = j & (Ns - 1);
                cx<R> a = src[j], b = src[j + M / 2];
                cx<R> w = tw[kk * (M / (2 * Ns))];
                b = cmul(b, w);
                const int d = ((j - kk) << 1) + kk;
                dst[d] = cadd(a, b);
                dst[d + Ns] = csub(a, b);
            }
            __syncthreads();
            cx<R> *t = src;
            src = dst;
            dst = t;
        }
        for (int k = threadIdx.x; k < K; k += blockDim.x) {
            const cx<R> zk = src[k], zn = src[(M - k) & (M - 1)];
            const cx<R> X[2] = {{(R)0.5 * (zk.re + zn.re), (R)0.5 * (zk.im - zn.im)},
                                {(R)0.5 * (zk.im + zn.im), (R)0.5 * (zn.re - zk.re)}};
            for (int j = 0; j < (two ? 2 : 1); ++j) {
                const int mj = m + j;
                const double S = L.psd_tf ? L.psd_tf[(size_t)k * Nt + mj] : L.psd0[k] * L.mu[mj];
                // a bin whose PSD is not positive and finite (DC or Nyquist may carry 0 or inf)
                // gets pixel 0 rather than inf or NaN; its template weight is 0 as well
                const double sc = L.keep[mj] != 0 && psd_ok(S) ? sqrt(2.0 * L.dt / ((double)M * w2 * S)) : 0.0;
                tile[(size_t)k * TB + tt + j] = cscale(X[j], (R)sc);
            }
        }
        __syncthreads();
    }
    // write out the tile
    const int ntb = min(TB, Nt - m0);
    if (L.out_layout == 0 || L.out_layout == 2) {
        for (int e = threadIdx.x; e < K * TB; e += blockDim.x) {
            const int k = e / TB, tt = e % TB;
            if (tt >= ntb) continue;
            cx<R> v = tile[e];
            size_t idx = L.out_layout == 0 ? ((size_t)c * K + k) * Nt + (m0 + tt)
                                           : ((size_t)k * Nt + (m0 + tt)) * L.C + c;
            reinterpret_cast<OutT *>(L.pix)[2 * idx] = (OutT)v.re;
            reinterpret_cast<OutT *>(L.pix)[2 * idx + 1] = (OutT)v.im;
        }
    } else {
        for (int e = threadIdx.x; e < K * TB; e += blockDim.x) {
            const int tt = e / K, k = e % K;
            if (tt >= ntb) continue;
            cx<R> v = tile[(size_t)k * TB + tt];
            size_t idx = ((size_t)c * Nt + (m0 + tt)) * K + k;
            reinterpret_cast<OutT *>(L.pix)[2 * idx] = (OutT)v.re;
            reinterpret_cast<OutT *>(L.pix)[2 * idx + 1] = (OutT)v.im;
        }
    }
}

// per-layer maximum |component| of an FP32 LAYER_MAJOR staging store
__global__ void k_layer_absmax(int C, int K, int Nt, const float *__restrict__ st, uint32_t *__restrict__ mx) {
    const int layer = blockIdx.x;  // c * K + k
    float v = 0.0f;
    const float *row = st + (size_t)layer * Nt * 2;
    for (int e = threadIdx.x; e < 2 * Nt; e += blockDim.x) v = fmaxf(v, fabsf(row[e]));
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    __shared__ float sh[16];
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        float m = 0.0f;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) m = fmaxf(m, sh[w]);
        mx[layer] = __float_as_uint(m);
    }
}

template <class Q>
__device__ __forceinline__ Q to_q(float v);
template <>
__device__ __forceinline__ __half to_q<__half>(float v) { return __float2half_rn(v); }
template <>
__device__ __forceinline__ __hip_bfloat16 to_q<__hip_bfloat16>(float v) { return __float2bfloat16(v); }
template <>
__device__ __forceinline__ int16_t to_q<int16_t>(float v) {
    // v = value / layer_scale lies in [-32767, 32767] up to rounding of the scale; nearest integer
    return (int16_t)fminf(fmaxf(rintf(v), -32767.0f), 32767.0f);
}
// Largest stored magnitude of each type: the floating types hold value / (layer max) in [-1, 1],
// the fixed-point type value / (layer max / 32767) on the integer grid.
template <class Q>
constexpr float q_full = 1.0f;
template <>
constexpr float q_full<int16_t> = 32767.0f;

template <class Q>
__global__ void k_quantize(int C, int K, int Nt, int layout, const float *__restrict__ st,
                           const uint32_t *__restrict__ mx, float *__restrict__ layer_scale, Q *__restrict__ out) {
    const int layer = blockIdx.y;
    const int c = layer / K, k = layer % K;
    float m = __uint_as_float(mx[layer]);
    float scale = m > 0.0f ? m / q_full<Q> : 1.0f;
    float inv = m > 0.0f ? q_full<Q> / m : 1.0f;
    if (blockIdx.x == 0 && threadIdx.x == 0) layer_scale[layer] = scale;
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < Nt; t += gridDim.x * blockDim.x) {
        const float *src = st + ((size_t)layer * Nt + t) * 2;
        size_t idx = layout == 0 ? ((size_t)layer * Nt + t)
                                 : (layout == 1 ? (((size_t)c * Nt + t) * K + k) : (((size_t)k * Nt + t) * C + c));
        out[2 * idx] = to_q<Q>(src[0] * inv);
        out[2 * idx + 1] = to_q<Q>(src[1] * inv);
    }
}

__global__ void k_weights(int K, int Nt, const double *__restrict__ psd0, const double *__restrict__ mu,
                          const uint8_t *__restrict__ keep, double *__restrict__ inv_asd, double *__restrict__ tw) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < K) inv_asd[i] = psd_ok(psd0[i]) ? 1.0 / sqrt(psd0[i]) : 0.0;
    if (i < Nt) tw[i] = keep[i] && psd_ok(mu[i]) ? 1.0 / sqrt(mu[i]) : 0.0;
}

// Template weights for a per-pixel PSD S_m(f_k) (psd[K][Nt]): one block per bin k forms
// S0_k = mean over the tranches of S_m(f_k) (fixed-order partial sums, then a fixed tree),
// u_k = 1/sqrt(S0_k) and rho_mk = sqrt(S0_k / S_m(f_k)); block 0 also writes w_m = keep_m.
__global__ __launch_bounds__(256) void k_weights_tf(int K, int Nt, const double *__restrict__ psd,
                                                   const uint8_t *__restrict__ keep, double *__restrict__ inv_asd,
                                                   double *__restrict__ tw, float *__restrict__ rho) {
    __shared__ double part[256];
    const int k = blockIdx.x;
    const double *row = psd + (size_t)k * Nt;
    double s = 0.0;
    for (int m = threadIdx.x; m < Nt; m += blockDim.x) s += row[m];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) part[threadIdx.x] += part[threadIdx.x + h];
        __syncthreads();
    }
    const double S0 = part[0] / (double)Nt;
    // a layer whose mean PSD is not positive and finite (DC or Nyquist may carry 0 or inf), or a
    // pixel whose own PSD is not, gets weight 0 (u_k or rho_mk), as its pixel is 0
    const bool ok0 = psd_ok(S0);
    if (threadIdx.x == 0) inv_asd[k] = ok0 ? 1.0 / sqrt(S0) : 0.0;
    for (int m = threadIdx.x; m < Nt; m += blockDim.x)
        rho[(size_t)k * Nt + m] = ok0 && psd_ok(row[m]) ? (float)sqrt(S0 / row[m]) : 0.0f;
    if (k == 0)
        for (int m = threadIdx.x; m < Nt; m += blockDim.x) tw[m] = keep[m] ? 1.0 : 0.0;
}

static double window_w2(int M, double alpha) {
    // mean of w^2 of the symmetric Tukey window (host side, FP64)
    if (alpha <= 0.0) return 1.0;
    double width = floor(alpha * (M - 1) / 2.0), s = 0.0;
    for (int n = 0; n < M; ++n) {
        int nn = n < M - 1 - n ? n : M - 1 - n;
        double w = 1.0;
        if ((double)nn <= width) w = 0.5 * (1.0 + cos(kPi * (-1.0 + 2.0 * nn / (alpha * (M - 1)))));
        s += w * w;
    }
    return s / M;
}

template <class R, class XT, class OutT, int TB>
static hipError_t run_fft(const TransformLaunch &L, TransformLaunch Lw, double w2, hipStream_t st) {
    const int M = L.M, K = M / 2 + 1;
    size_t shmem = sizeof(cx<R>) * (2 * (size_t)M + M / 2 + (size_t)K * TB) + sizeof(R) * M;
    static bool attr_set = false;
    if (!attr_set) {
        (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_transform<R, XT, OutT, TB>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        attr_set = true;
    }
    dim3 grid((unsigned)((L.Nt + TB - 1) / TB), (unsigned)L.C);
    hipLaunchKernelGGL((k_transform<R, XT, OutT, TB>), grid, dim3(256), shmem, st, Lw, w2);
    return hipGetLastError();
}

hipError_t launch_transform(const TransformLaunch &L, hipStream_t st) {
    const int K = L.M / 2 + 1;
    const double w2 = window_w2(L.M, L.alpha);
    int nw = K > L.Nt ? K : L.Nt;
    if (L.psd_tf)
        hipLaunchKernelGGL(k_weights_tf, dim3(K), dim3(256), 0, st, K, L.Nt, L.psd_tf, L.keep, L.inv_asd,
                           L.tranche_w, L.rho);
    else
        hipLaunchKernelGGL(k_weights, dim3((nw + 255) / 256), dim3(256), 0, st, K, L.Nt, L.psd0, L.mu, L.keep,
                           L.inv_asd, L.tranche_w);
    const bool q16 = L.out_dtype == 2 || L.out_dtype == 3 || L.out_dtype == 4;
    TransformLaunch Lw = L;
    hipError_t e;
    // The FFT runs in FP64 whenever the tile fits in LDS (M <= 2048): whitening divides by
    // sqrt(S0), which near the TDI nulls is ~1e5 smaller than at low frequency, so FP32 FFT
    // rounding (set by the red low-frequency power) would be amplified there.
    const bool big = L.M > 2048;
    if (q16) {
        // FP32 LAYER_MAJOR staging, then per-layer scale and quantisation
        Lw.pix = L.ws;
        Lw.out_layout = 0;
        if (L.x_dtype == 0)
            e = big ? run_fft<float, double, float, 2>(L, Lw, w2, st) : run_fft<double, double, float, 2>(L, Lw, w2, st);
        else
            e = big ? run_fft<float, float, float, 2>(L, Lw, w2, st) : run_fft<double, float, float, 2>(L, Lw, w2, st);
        if (e != hipSuccess) return e;
        size_t st_bytes = sizeof(float) * 2 * (size_t)L.C * K * L.Nt;
        st_bytes = (st_bytes + 255) / 256 * 256;
        uint32_t *mx = reinterpret_cast<uint32_t *>(reinterpret_cast<char *>(L.ws) + st_bytes);
        hipLaunchKernelGGL(k_layer_absmax, dim3(L.C * K), dim3(256), 0, st, L.C, K, L.Nt,
                           reinterpret_cast<const float *>(L.ws), mx);
        dim3 g((unsigned)((L.Nt + 255) / 256 > 8 ? 8 : (L.Nt + 255) / 256), (unsigned)(L.C * K));
        if (L.out_dtype == 4)
            hipLaunchKernelGGL(k_quantize<int16_t>, g, dim3(256), 0, st, L.C, K, L.Nt, L.out_layout,
                               reinterpret_cast<const float *>(L.ws), mx, L.layer_scale,
                               reinterpret_cast<int16_t *>(L.pix));
        else if (L.out_dtype == 3)
            hipLaunchKernelGGL(k_quantize<__half>, g, dim3(256), 0, st, L.C, K, L.Nt, L.out_layout,
                               reinterpret_cast<const float *>(L.ws), mx, L.layer_scale,
                               reinterpret_cast<__half *>(L.pix));
        else
            hipLaunchKernelGGL(k_quantize<__hip_bfloat16>, g, dim3(256), 0, st, L.C, K, L.Nt, L.out_layout,
                               reinterpret_cast<const float *>(L.ws), mx, L.layer_scale,
                               reinterpret_cast<__hip_bfloat16 *>(L.pix));
        return hipGetLastError();
    }
    if (L.out_dtype == 0) return big ? hipErrorInvalidValue : run_fft<double, double, double, 2>(L, Lw, w2, st);
    if (L.x_dtype == 0)
        return big ? run_fft<float, double, float, 2>(L, Lw, w2, st) : run_fft<double, double, float, 2>(L, Lw, w2, st);
    return big ? run_fft<float, float, float, 2>(L, Lw, w2, st) : run_fft<double, float, float, 2>(L, Lw, w2, st);
}

}  // namespace tfsc
