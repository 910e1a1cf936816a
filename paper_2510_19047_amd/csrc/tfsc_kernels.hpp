// Internal launch descriptors shared by the C ABI layer and the kernel files.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tfsc {

// Layout of the statistic workspace's tail: the WAVE schedule's uint32 work counter at
// +0, the FP64 weight scale at +kTailScale.
constexpr int kTailScale = 64;

// Geometry tables in the statistic workspace: 18 FP64 rows of Nt values, then (256-byte
// aligned) the FP32 copy of the 9 arm-vector rows.
inline size_t geo64_bytes(int Nt) { return (sizeof(double) * 18 * (size_t)Nt + 255) / 256 * 256; }
inline size_t geo32_bytes(int Nt) { return (sizeof(float) * 9 * (size_t)Nt + 255) / 256 * 256; }
inline float *geo32_of(const double *geo, int Nt) {
    return reinterpret_cast<float *>(reinterpret_cast<char *>(const_cast<double *>(geo)) + geo64_bytes(Nt));
}

struct LayoutLaunch {
    int64_t n;
    const double *mc, *eta, *f0, *ct, *ci;
    const double *ln_mc;  // the bank given in ln Mc (mc unused), else NULL
    int nseg_fixed;
    int32_t *nseg;
    int64_t *seg_offset;
    int64_t *block_sums;  // workspace, ceil(n / 256) entries
};

struct StatLaunch {
    int M, Nt, C;
    double dt;
    int pix_dtype;  // tfsc_dtype
    int layout;     // tfsc_layout
    int precision;  // 0 FP64, 1 FP32
    int schedule;   // 0 THREAD, 1 WAVE
    int n_groups, block_waves;
    const void *pix;
    const float *layer_scale;
    const double *inv_asd, *tranche_w, *geo;
    const float *rho;       // [K][Nt] per-pixel weight factor, NULL for a separable PSD
    const double *links;    // [6][Nt] link light times (unequal arms), NULL for equal arms
    int tdi2;               // with links: second-generation TDI combinations
    const double *u_scale;  // device scalar written by launch_weight_scale
    int64_t n;
    const double *mc, *eta, *f0, *ct, *phi, *psi, *ci;
    const double *ln_mc;  // the bank given in ln Mc: the entry point fills mc (a workspace table) from it
    const int32_t *nseg;
    const int64_t *seg_offset;
    const int32_t *order;
    double *seg_terms, *stat, *seg_zn;
    int32_t *flags;
    int32_t *n_active;
    uint32_t *counter;
    // several realisations (launch_statistic_multi only)
    int n_real;
    int64_t real_stride;  // bytes between realisation stores
    int64_t seg_stride;   // elements between realisation planes of seg_terms
    int multi_group;      // realisations sharing one pass over the bank: 1, 2, 4 or 8
};

constexpr int kMultiGroupDefault = 8;
constexpr int kMaxRealisations = 64;

struct VjpLaunch {
    StatLaunch s;  // seg_terms / stat / flags unused
    const double *seg_zn;
    const double *g_stat, *g_seg;
    double *g_params;
};

// Processing order: templates grouped by the frequency bin of f0, then by ln Mc in kOrderMcClasses classes
// over [kOrderLnMcLo, kOrderLnMcHi) (clamped at the ends).
constexpr int kOrderMcClasses = 256;
constexpr double kOrderLnMcLo = -0.6931471805599453;  // ln 0.5
constexpr double kOrderLnMcHi = 6.214608098422191;    // ln 500

struct OrderLaunch {
    int M;
    double dt;
    int64_t n;
    const double *mc, *eta, *f0, *ct, *ci;
    const double *ln_mc;
    int32_t *order;
    uint32_t *ws;  // 2 nb + ceil(nb / 1024) counters, nb = (M/2 + 1) kOrderMcClasses + 1
};

struct FollowLaunch {
    int Nt;
    double dT;
    int64_t n;
    double *mc, *f0, *ct, *phi, *psi;  // updated in place
    double *ln_mc;                     // updated in place instead of mc when the bank is given in ln Mc
    const double *eta, *ci;
    const int32_t *nseg;
    const double *stat, *g_params;
    double *state;  // [n][16]
    double lr_scale;
    int step;
};

struct TransformLaunch {
    int M, Nt, C;
    double dt, alpha;
    const void *x;
    int x_dtype;
    const double *psd0, *mu;
    const double *psd_tf;  // [K][Nt] S_m(f_k) for a general per-pixel PSD (then psd0, mu unused), else NULL
    const uint8_t *keep;
    int out_dtype, out_layout;
    void *pix;
    float *layer_scale;
    double *inv_asd, *tranche_w;
    float *rho;  // written when psd_tf is set
    void *ws;  // FP32 staging for 16-bit outputs
};

hipError_t launch_layout(const LayoutLaunch &L, hipStream_t st);
hipError_t launch_geometry(int Nt, double dT, const double *orbit, double *geo, hipStream_t st);
hipError_t launch_orbit_positions(int Nt, double dT, double *out, hipStream_t st);
hipError_t launch_link_lengths(int Nt, double dT, const double *orbit, double *out, hipStream_t st);
hipError_t launch_statistic_interleaved(const StatLaunch &L, hipStream_t st);
hipError_t launch_interleave(int64_t cells, int C, int K, int NR, int r, int elem_bytes, const void *src,
                             const float *src_scale, void *dst, float *dst_scale, hipStream_t st);
hipError_t launch_exp_mc(int64_t n, const double *ln_mc, double *mc, hipStream_t st);
hipError_t launch_weight_scale(int K, const double *inv_asd, double *scale_out, hipStream_t st);
hipError_t launch_statistic(const StatLaunch &L, hipStream_t st);
hipError_t launch_statistic_accurate(const StatLaunch &L, hipStream_t st);
hipError_t launch_statistic_links(const StatLaunch &L, hipStream_t st);
constexpr int kMaxHarmonics = 4;
hipError_t launch_statistic_harmonics(const StatLaunch &L, int n_harm, const int *harm, const double *amp,
                                      hipStream_t st);
hipError_t launch_statistic_multi(const StatLaunch &L, hipStream_t st);
hipError_t launch_vjp(const VjpLaunch &L, hipStream_t st);
hipError_t launch_transform(const TransformLaunch &L, hipStream_t st);
hipError_t launch_follow_step(const FollowLaunch &L, hipStream_t st);
hipError_t launch_order(const OrderLaunch &L, hipStream_t st);
hipError_t launch_tile_max(const double *stat, const int32_t *tile, int64_t n, int32_t n_tiles, double *tile_max,
                           int64_t *tile_arg, hipStream_t st);
hipError_t launch_track(int64_t n, int M, int Nt, double dt, const double *mc, const double *ln_mc, const double *eta,
                        const double *f0, const double *ct, const double *ci, double *out, hipStream_t st);

}  // namespace tfsc
