// C ABI of libtfsc.so: argument checks, workspace carving and launches.
#include <math.h>
#include <string.h>

#include <map>
#include <mutex>
#include <string>

#include "../../include/tfsc.h"
#include "tfsc_kernels.hpp"

// Device scratch of tfsc_bank_statistic_noalloc: the statistic workspace (geometry tables, work
// counter, weight scale) for grids of up to TFSC_NOALLOC_MAX_TRANCHES tranches.  Each device holds
// its own copy for the life of the process; host code reaches it only through the address that
// hipGetSymbolAddress returns on that device (scratch_on_device below), never through the name.
constexpr size_t kScratchBytes = TFSC_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

int device_cus() {
    static int cached[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    if (cached[dev] == 0) {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            cus = 256;
        cached[dev] = cus;
    }
    return cached[dev];
}

bool pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

tfsc_status check_grid(const tfsc_grid *g) {
    if (!g) return TFSC_ERR_ARG;
    if (g->n_channels < 1 || g->n_channels > 3) return TFSC_ERR_SHAPE;
    if (g->tranche_len < 64 || g->tranche_len > 4096 || !pow2(g->tranche_len)) return TFSC_ERR_SHAPE;
    if (g->n_tranches < 1) return TFSC_ERR_SHAPE;
    if (g->n_fresnel != 21) return TFSC_ERR_UNSUPPORTED;
    if (!(g->dt > 0.0)) return TFSC_ERR_ARG;
    if (!(g->tukey_alpha >= 0.0 && g->tukey_alpha <= 1.0)) return TFSC_ERR_ARG;
    return TFSC_OK;
}

tfsc_status check_bank(const tfsc_bank *b) {
    if (!b) return TFSC_ERR_ARG;
    if (b->n < 0 || b->n > 0x7fffffffLL) return TFSC_ERR_SHAPE;
    // exactly one of mc and ln_mc
    if (b->n > 0 && ((!b->mc) == (!b->ln_mc))) return TFSC_ERR_ARG;
    if (b->n > 0 && (!b->eta || !b->f0 || !b->cos_theta || !b->phi || !b->psi || !b->cos_iota)) return TFSC_ERR_ARG;
    return TFSC_OK;
}

// BF16, F16 and I16 stores: 16-bit values with a per-layer FP32 scale
inline bool is_16bit(int d) { return d == TFSC_BF16 || d == TFSC_F16 || d == TFSC_I16; }

tfsc_status check_pixels(const tfsc_pixels *p, bool need_data) {
    if (!p) return TFSC_ERR_ARG;
    if (p->dtype < TFSC_F64 || p->dtype > TFSC_I16) return TFSC_ERR_DTYPE;
    if (p->layout != TFSC_LAYER_MAJOR && p->layout != TFSC_TRANCHE_MAJOR && p->layout != TFSC_LAYER_MAJOR_CI)
        return TFSC_ERR_ARG;
    if (need_data && !p->pix) return TFSC_ERR_ARG;
    if (!p->inv_asd || !p->tranche_w) return TFSC_ERR_ARG;
    if (is_16bit(p->dtype) && !p->layer_scale) return TFSC_ERR_ARG;
    if (p->tdi_generation < 0 || p->tdi_generation > 2) return TFSC_ERR_ARG;
    if (p->tdi_generation == 2 && !p->links) return TFSC_ERR_UNSUPPORTED;
    return TFSC_OK;
}

struct Resolved {
    int precision, schedule, block_waves, groups_per_cu, fresnel;
    const int32_t *order;
};

// Launch shapes chosen by tfsc_tune_statistic, per tune key, for the life of the process.
struct TuneTable {
    std::mutex mu;
    std::map<std::string, std::pair<int, int>> shape;
};
TuneTable &tune_table() {
    static TuneTable t;
    return t;
}

tfsc_status resolve_options(const tfsc_options *o, const tfsc_pixels *p, Resolved &r) {
    r.precision = o ? o->precision : TFSC_F64;
    r.schedule = o ? o->schedule : TFSC_SCHED_WAVE;
    r.block_waves = (o && o->block_waves > 0) ? o->block_waves : 4;
    r.groups_per_cu = (o && o->groups_per_cu > 0) ? o->groups_per_cu : 4;
    r.order = o ? o->order : nullptr;
    r.fresnel = o ? o->fresnel : TFSC_FRESNEL_PAPER;
    if (o && o->tune_key && o->block_waves <= 0 && o->groups_per_cu <= 0) {
        TuneTable &t = tune_table();
        std::lock_guard<std::mutex> lock(t.mu);
        auto it = t.shape.find(o->tune_key);
        if (it != t.shape.end()) {
            r.block_waves = it->second.first;
            r.groups_per_cu = it->second.second;
        }
    }
    if (r.fresnel != TFSC_FRESNEL_PAPER && r.fresnel != TFSC_FRESNEL_ACCURATE) return TFSC_ERR_ARG;
    if (r.precision != TFSC_F64 && r.precision != TFSC_F32) return TFSC_ERR_DTYPE;
    if (r.schedule != TFSC_SCHED_THREAD && r.schedule != TFSC_SCHED_WAVE) return TFSC_ERR_ARG;
    // the WAVE and VJP kernels are compiled for at most 256 threads (4 waves) per block
    if (r.block_waves > 4 || r.groups_per_cu > 64) return TFSC_ERR_ARG;
    if (p) {
        if (r.precision == TFSC_F64 && is_16bit(p->dtype)) return TFSC_ERR_DTYPE;
        if (r.precision == TFSC_F32 && p->dtype == TFSC_F64) return TFSC_ERR_DTYPE;
        if (r.schedule == TFSC_SCHED_WAVE && p->layout == TFSC_TRANCHE_MAJOR) return TFSC_ERR_UNSUPPORTED;
    }
    return TFSC_OK;
}

size_t pixel_store_bytes(const tfsc_grid *g, const tfsc_pixels *p) {
    const size_t b = p->dtype == TFSC_F64 ? 16 : (p->dtype == TFSC_F32 ? 8 : 4);
    return b * (size_t)g->n_channels * (size_t)(g->tranche_len / 2 + 1) * (size_t)g->n_tranches;
}

size_t geo_bytes(int Nt) { return tfsc::geo64_bytes(Nt) + tfsc::geo32_bytes(Nt); }

// Statistic and VJP workspace: the geometry tables, the tail (work counter, weight scale) and, for a
// bank given in ln Mc, a table of the chirp masses exp(ln Mc) formed once per call, so the
// kernels read Mc as they read every other parameter.
size_t stat_ws_bytes(const tfsc_grid *g, int64_t n, bool log_mc) {
    return geo_bytes(g->n_tranches) + kAlign + (log_mc ? align_up(sizeof(double) * (size_t)n) : 0);
}

size_t ws_bytes_for(const tfsc_grid *g, int64_t n, int which) {
    switch (which) {
        case TFSC_WS_LAYOUT:
            return align_up(sizeof(int64_t) * (size_t)((n + 255) / 256 + 1));
        case TFSC_WS_STATISTIC:
        case TFSC_WS_VJP:
            return stat_ws_bytes(g, n, true);
        case TFSC_WS_ORDER:
        {
            const size_t nb = (size_t)(g->tranche_len / 2 + 1) * tfsc::kOrderMcClasses + 1;
            return align_up(sizeof(uint32_t) * (2 * nb + (nb + 1023) / 1024));
        }
        case TFSC_WS_TRANSFORM: {
            size_t K = (size_t)g->tranche_len / 2 + 1;
            return align_up(sizeof(float) * 2 * (size_t)g->n_channels * K * (size_t)g->n_tranches) +
                   align_up(sizeof(uint32_t) * (size_t)g->n_channels * K);
        }
    }
    return 0;
}

tfsc_status hip_status(hipError_t e) { return e == hipSuccess ? TFSC_OK : TFSC_ERR_HIP; }

// The device address of `scratch` on the current device, looked up once per device (with that
// device current) and kept; NULL if the lookup fails.
void *scratch_on_device() {
    constexpr int kMaxDevices = 64;
    static void *addr[kMaxDevices] = {nullptr};
    static bool done[kMaxDevices] = {false};
    static std::mutex mu;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(mu);
    if (!done[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
        addr[dev] = p;
        done[dev] = true;
    }
    return addr[dev];
}

tfsc::StatLaunch stat_launch(const tfsc_grid *grid, const tfsc_pixels *pix, const tfsc_bank *bank,
                             const tfsc_segments *seg, const Resolved &r, void *ws) {
    tfsc::StatLaunch L;
    memset(&L, 0, sizeof(L));
    L.M = grid->tranche_len;
    L.Nt = grid->n_tranches;
    L.C = grid->n_channels;
    L.dt = grid->dt;
    L.pix_dtype = pix->dtype;
    L.layout = pix->layout;
    L.precision = r.precision == TFSC_F64 ? 0 : 1;
    L.schedule = r.schedule;
    L.block_waves = r.block_waves;
    L.n_groups = device_cus() * r.groups_per_cu;
    L.pix = pix->pix;
    L.layer_scale = pix->layer_scale;
    L.inv_asd = pix->inv_asd;
    L.tranche_w = pix->tranche_w;
    L.rho = pix->rho;
    L.links = pix->links;
    L.tdi2 = pix->links && pix->tdi_generation == 2;
    L.geo = reinterpret_cast<const double *>(ws);
    L.n = bank->n;
    L.mc = bank->mc;
    L.eta = bank->eta;
    L.f0 = bank->f0;
    L.ct = bank->cos_theta;
    L.phi = bank->phi;
    L.psi = bank->psi;
    L.ci = bank->cos_iota;
    L.ln_mc = bank->ln_mc;
    L.nseg = seg->nseg;
    L.seg_offset = seg->seg_offset;
    L.order = r.order;
    char *tail = reinterpret_cast<char *>(ws) + geo_bytes(grid->n_tranches);
    L.counter = reinterpret_cast<uint32_t *>(tail);
    L.u_scale = reinterpret_cast<const double *>(tail + tfsc::kTailScale);
    if (bank->ln_mc) L.mc = reinterpret_cast<const double *>(tail + kAlign);  // filled by prepare_launch
    return L;
}

// Per-call tables the kernels read: the geometry of the orbit, the weight scale and, for a bank
// given in ln Mc, the chirp masses.
hipError_t prepare_launch(const tfsc_grid *grid, const tfsc_pixels *pix, const tfsc::StatLaunch &L, void *ws,
                          hipStream_t st) {
    hipError_t e = tfsc::launch_geometry(grid->n_tranches, (double)grid->tranche_len * grid->dt, pix->orbit,
                                         reinterpret_cast<double *>(ws), st);
    if (e != hipSuccess) return e;
    e = tfsc::launch_weight_scale(grid->tranche_len / 2 + 1, pix->inv_asd, const_cast<double *>(L.u_scale), st);
    if (e != hipSuccess || !L.ln_mc) return e;
    return tfsc::launch_exp_mc(L.n, L.ln_mc, const_cast<double *>(L.mc), st);
}

}  // namespace

extern "C" {

int tfsc_abi_version(void) { return TFSC_ABI_VERSION; }

const char *tfsc_status_string(int s) {
    switch (s) {
        case TFSC_OK: return "ok";
        case TFSC_ERR_ARG: return "invalid argument (null pointer or out-of-range value)";
        case TFSC_ERR_SHAPE: return "inconsistent or unsupported sizes";
        case TFSC_ERR_DTYPE: return "unsupported element type or precision combination";
        case TFSC_ERR_WORKSPACE: return "workspace missing or too small";
        case TFSC_ERR_UNSUPPORTED: return "request not supported by the library";
        case TFSC_ERR_HIP: return "HIP runtime error";
        case TFSC_ERR_SCRATCH: return "problem larger than the library's static device scratch";
    }
    return "unknown status";
}

size_t tfsc_workspace_bytes(const tfsc_grid *grid, int64_t n_templates, const tfsc_options *opt, int which) {
    (void)opt;
    if (check_grid(grid) != TFSC_OK || n_templates < 0) return 0;
    return ws_bytes_for(grid, n_templates, which);
}

tfsc_status tfsc_segment_layout(const tfsc_grid *grid, const tfsc_bank *bank, tfsc_segments *seg, void *ws,
                                size_t ws_bytes, void *stream) {
    tfsc_status s;
    if ((s = check_grid(grid)) != TFSC_OK) return s;
    if ((s = check_bank(bank)) != TFSC_OK) return s;
    if (!seg || !seg->seg_offset || (bank->n > 0 && !seg->nseg)) return TFSC_ERR_ARG;
    if (seg->nseg_fixed < 0 || seg->nseg_fixed > (1 << 20)) return TFSC_ERR_ARG;
    if (!ws || ws_bytes < ws_bytes_for(grid, bank->n, TFSC_WS_LAYOUT)) return TFSC_ERR_WORKSPACE;
    tfsc::LayoutLaunch L;
    L.n = bank->n;
    L.mc = bank->mc;
    L.eta = bank->eta;
    L.f0 = bank->f0;
    L.ct = bank->cos_theta;
    L.ci = bank->cos_iota;
    L.ln_mc = bank->ln_mc;
    L.nseg_fixed = seg->nseg_fixed;
    L.nseg = seg->nseg;
    L.seg_offset = seg->seg_offset;
    L.block_sums = reinterpret_cast<int64_t *>(ws);
    return hip_status(tfsc::launch_layout(L, reinterpret_cast<hipStream_t>(stream)));
}

tfsc_status tfsc_bank_statistic(const tfsc_grid *grid, const tfsc_pixels *pix, const tfsc_bank *bank,
                                const tfsc_segments *seg, const tfsc_options *opt, double *seg_terms, double *stat,
                                double *seg_zn, int32_t *flags, int32_t *n_active, void *ws, size_t ws_bytes,
                                void *stream) {
    tfsc_status s;
    if ((s = check_grid(grid)) != TFSC_OK) return s;
    if ((s = check_bank(bank)) != TFSC_OK) return s;
    if ((s = check_pixels(pix, bank->n > 0)) != TFSC_OK) return s;
    if (!seg || (bank->n > 0 && (!seg->nseg || !seg->seg_offset))) return TFSC_ERR_ARG;
    Resolved r;
    if ((s = resolve_options(opt, pix, r)) != TFSC_OK) return s;
    if (bank->n > 0 && (!seg_terms || !stat || !flags)) return TFSC_ERR_ARG;
    if (!ws || ws_bytes < stat_ws_bytes(grid, bank->n, bank->ln_mc != nullptr)) return TFSC_ERR_WORKSPACE;
    if (r.schedule == TFSC_SCHED_WAVE && pixel_store_bytes(grid, pix) > 0xffffffffull) return TFSC_ERR_UNSUPPORTED;
    if (pix->rho && r.schedule == TFSC_SCHED_WAVE && pix->dtype != TFSC_F64 && pix->dtype != TFSC_F32)
        return TFSC_ERR_UNSUPPORTED;
    if (r.fresnel == TFSC_FRESNEL_ACCURATE &&
        (pix->rho || !((pix->dtype == TFSC_F64 && r.precision == TFSC_F64) ||
                       (pix->dtype == TFSC_F32 && r.precision == TFSC_F32))))
        return TFSC_ERR_UNSUPPORTED;
    if (pix->links && (pix->rho || r.fresnel != TFSC_FRESNEL_PAPER ||
                       !((pix->dtype == TFSC_F64 && r.precision == TFSC_F64) ||
                         (pix->dtype == TFSC_F32 && r.precision == TFSC_F32))))
        return TFSC_ERR_UNSUPPORTED;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (bank->n == 0) return TFSC_OK;
    tfsc::StatLaunch L = stat_launch(grid, pix, bank, seg, r, ws);
    if (prepare_launch(grid, pix, L, ws, st) != hipSuccess) return TFSC_ERR_HIP;
    L.seg_terms = seg_terms;
    L.stat = stat;
    L.seg_zn = seg_zn;
    L.flags = flags;
    L.n_active = n_active;
    if (r.fresnel == TFSC_FRESNEL_ACCURATE) return hip_status(tfsc::launch_statistic_accurate(L, st));
    if (pix->links) return hip_status(tfsc::launch_statistic_links(L, st));
    return hip_status(tfsc::launch_statistic(L, st));
}

tfsc_status tfsc_bank_statistic_noalloc(const tfsc_grid *grid, const tfsc_pixels *pix, const tfsc_bank *bank,
                                        const tfsc_segments *seg, const tfsc_options *opt, double *seg_terms,
                                        double *stat, double *seg_zn, int32_t *flags, int32_t *n_active,
                                        void *stream) {
    tfsc_status s;
    if ((s = check_grid(grid)) != TFSC_OK) return s;
    const size_t need = stat_ws_bytes(grid, bank ? bank->n : 0, bank && bank->ln_mc);
    if (grid->n_tranches > TFSC_NOALLOC_MAX_TRANCHES || need > kScratchBytes) return TFSC_ERR_SCRATCH;
    void *ws = scratch_on_device();
    if (!ws) return TFSC_ERR_HIP;
    return tfsc_bank_statistic(grid, pix, bank, seg, opt, seg_terms, stat, seg_zn, flags, n_active, ws, need,
                               stream);
}

tfsc_status tfsc_bank_statistic_multi(const tfsc_grid *grid, const tfsc_pixels *pix, int32_t n_real,
                                      int64_t real_stride, int32_t group, const tfsc_bank *bank,
                                      const tfsc_segments *seg, const tfsc_options *opt, int64_t seg_stride,
                                      double *seg_terms, double *stat, int32_t *flags, int32_t *n_active, void *ws,
                                      size_t ws_bytes, void *stream) {
    tfsc_status s;
    if ((s = check_grid(grid)) != TFSC_OK) return s;
    if ((s = check_bank(bank)) != TFSC_OK) return s;
    if ((s = check_pixels(pix, bank->n > 0)) != TFSC_OK) return s;
    if (!seg || (bank->n > 0 && (!seg->nseg || !seg->seg_offset))) return TFSC_ERR_ARG;
    if (n_real < 1 || n_real > tfsc::kMaxRealisations || seg_stride < 0) return TFSC_ERR_ARG;
    if (group != 0 && group != 1 && group != 2 && group != 4 && group != 8) return TFSC_ERR_ARG;
    Resolved r;
    if ((s = resolve_options(opt, pix, r)) != TFSC_OK) return s;
    if (r.schedule != TFSC_SCHED_WAVE || pix->layout == TFSC_TRANCHE_MAJOR || grid->n_channels == 3 ||
        r.fresnel != TFSC_FRESNEL_PAPER || pix->links)
        return TFSC_ERR_UNSUPPORTED;
    const bool interleaved = real_stride == 0;
    if (!(pix->dtype == TFSC_F32 && r.precision == TFSC_F32) && !(pix->dtype == TFSC_F64 && r.precision == TFSC_F64) &&
        !(interleaved && pix->dtype == TFSC_I16 && r.precision == TFSC_F32))
        return TFSC_ERR_DTYPE;
    const uint64_t one = pixel_store_bytes(grid, pix);
    if (interleaved) {
        // realisations interleaved cell by cell: FP32, channel-interleaved, 2 or 4 of them, no rho
        if (pix->layout != TFSC_LAYER_MAJOR_CI || (pix->dtype != TFSC_F32 && pix->dtype != TFSC_I16) ||
            r.precision != TFSC_F32 || pix->rho || (n_real != 2 && n_real != 4) || (group != 0 && group != n_real))
            return TFSC_ERR_UNSUPPORTED;
        if (one * (uint64_t)n_real > 0xffffffffull) return TFSC_ERR_UNSUPPORTED;
    } else {
        if (real_stride < 0 || (uint64_t)real_stride < one || real_stride % 16 != 0) return TFSC_ERR_SHAPE;
        if ((uint64_t)real_stride * (uint64_t)n_real > 0xffffffffull) return TFSC_ERR_UNSUPPORTED;
    }
    if (bank->n > 0 && (!seg_terms || !stat || !flags)) return TFSC_ERR_ARG;
    if (!ws || ws_bytes < stat_ws_bytes(grid, bank->n, bank->ln_mc != nullptr)) return TFSC_ERR_WORKSPACE;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (bank->n == 0) return TFSC_OK;
    tfsc::StatLaunch L = stat_launch(grid, pix, bank, seg, r, ws);
    if (prepare_launch(grid, pix, L, ws, st) != hipSuccess) return TFSC_ERR_HIP;
    L.seg_terms = seg_terms;
    L.stat = stat;
    L.flags = flags;
    L.n_active = n_active;
    L.n_real = n_real;
    L.real_stride = real_stride;
    L.seg_stride = seg_stride;
    L.multi_group = group == 0 ? tfsc::kMultiGroupDefault : group;
    if (interleaved) return hip_status(tfsc::launch_statistic_interleaved(L, st));
    return hip_status(tfsc::launch_statistic_multi(L, st));
}

tfsc_status tfsc_interleave_store(const tfsc_grid *grid, const tfsc_pixels *src, int32_t n_real, int32_t r,
                                  tfsc_pixels *dst, void *stream) {
    tfsc_status s;
    if ((s = check_grid(grid)) != TFSC_OK) return s;
    if (!src || !src->pix || !dst || !dst->pix) return TFSC_ERR_ARG;
    if ((src->dtype != TFSC_F32 && src->dtype != TFSC_I16) || dst->dtype != src->dtype) return TFSC_ERR_DTYPE;
    if (src->layout != TFSC_LAYER_MAJOR_CI || dst->layout != TFSC_LAYER_MAJOR_CI) return TFSC_ERR_UNSUPPORTED;
    if (src->dtype == TFSC_I16 && (!src->layer_scale || !dst->layer_scale)) return TFSC_ERR_ARG;
    if (n_real < 1 || n_real > tfsc::kMaxRealisations || r < 0 || r >= n_real) return TFSC_ERR_ARG;
    const int K = grid->tranche_len / 2 + 1;
    const int64_t cells = (int64_t)K * grid->n_tranches;
    const bool i16 = src->dtype == TFSC_I16;
    return hip_status(tfsc::launch_interleave(cells, grid->n_channels, K, n_real, r, i16 ? 4 : 8, src->pix,
                                              i16 ? src->layer_scale : nullptr, dst->pix,
                                              i16 ? dst->layer_scale : nullptr, reinterpret_cast<hipStream_t>(stream)));
}

tfsc_status tfsc_statistic_vjp(const tfsc_grid *grid, const tfsc_pixels *pix, const tfsc_bank *bank,
                               const tfsc_segments *seg, const tfsc_options *opt, const double *seg_zn,
                               const double *g_stat, const double *g_seg, double *g_params, void *ws,
                               size_t ws_bytes, void *stream) {
    tfsc_status s;
    if ((s = check_grid(grid)) != TFSC_OK) return s;
    if ((s = check_bank(bank)) != TFSC_OK) return s;
    if ((s = check_pixels(pix, bank->n > 0)) != TFSC_OK) return s;
    if (!seg || (bank->n > 0 && (!seg->nseg || !seg->seg_offset))) return TFSC_ERR_ARG;
    // Either arithmetic reads every pixel type and layout (no pixel check against the precision).
    Resolved r;
    if ((s = resolve_options(opt, nullptr, r)) != TFSC_OK) return s;
    if (r.fresnel != TFSC_FRESNEL_PAPER || pix->links) return TFSC_ERR_UNSUPPORTED;
    if (bank->n > 0 && (!seg_zn || !g_params || (!g_stat && !g_seg))) return TFSC_ERR_ARG;
    if (!ws || ws_bytes < stat_ws_bytes(grid, bank->n, bank->ln_mc != nullptr)) return TFSC_ERR_WORKSPACE;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (bank->n == 0) return TFSC_OK;
    tfsc::VjpLaunch V;
    V.s = stat_launch(grid, pix, bank, seg, r, ws);
    if (prepare_launch(grid, pix, V.s, ws, st) != hipSuccess) return TFSC_ERR_HIP;
    V.seg_zn = seg_zn;
    V.g_stat = g_stat;
    V.g_seg = g_seg;
    V.g_params = g_params;
    return hip_status(tfsc::launch_vjp(V, st));
}

tfsc_status tfsc_processing_order(const tfsc_grid *grid, const tfsc_bank *bank, int32_t *order, void *ws,
                                  size_t ws_bytes, void *stream) {
    tfsc_status s;
    if ((s = check_grid(grid)) != TFSC_OK) return s;
    if ((s = check_bank(bank)) != TFSC_OK) return s;
    if (bank->n > 0 && !order) return TFSC_ERR_ARG;
    if (!ws || ws_bytes < ws_bytes_for(grid, bank->n, TFSC_WS_ORDER)) return TFSC_ERR_WORKSPACE;
    tfsc::OrderLaunch L;
    L.M = grid->tranche_len;
    L.dt = grid->dt;
    L.n = bank->n;
    L.mc = bank->mc;
    L.eta = bank->eta;
    L.f0 = bank->f0;
    L.ct = bank->cos_theta;
    L.ci = bank->cos_iota;
    L.ln_mc = bank->ln_mc;
    L.order = order;
    L.ws = reinterpret_cast<uint32_t *>(ws);
    return hip_status(tfsc::launch_order(L, reinterpret_cast<hipStream_t>(stream)));
}

tfsc_status tfsc_follow_up_step(const tfsc_grid *grid, tfsc_bank *bank, const tfsc_segments *seg,
                                const double *stat, const double *g_params, double *state, double lr_scale,
                                int step, void *stream) {
    tfsc_status s;
    if ((s = check_grid(grid)) != TFSC_OK) return s;
    if ((s = check_bank(bank)) != TFSC_OK) return s;
    if (step < 1 || !(lr_scale >= 0.0) || !isfinite(lr_scale)) return TFSC_ERR_ARG;
    if (bank->n == 0) return TFSC_OK;
    if (!seg || !seg->nseg || !stat || !g_params || !state) return TFSC_ERR_ARG;
    tfsc::FollowLaunch L;
    L.Nt = grid->n_tranches;
    L.dT = (double)grid->tranche_len * grid->dt;
    L.n = bank->n;
    L.mc = const_cast<double *>(bank->mc);
    L.ln_mc = const_cast<double *>(bank->ln_mc);
    L.f0 = const_cast<double *>(bank->f0);
    L.ct = const_cast<double *>(bank->cos_theta);
    L.phi = const_cast<double *>(bank->phi);
    L.psi = const_cast<double *>(bank->psi);
    L.eta = bank->eta;
    L.ci = bank->cos_iota;
    L.nseg = seg->nseg;
    L.stat = stat;
    L.g_params = g_params;
    L.state = state;
    L.lr_scale = lr_scale;
    L.step = step;
    return hip_status(tfsc::launch_follow_step(L, reinterpret_cast<hipStream_t>(stream)));
}

tfsc_status tfsc_tile_max(const double *stat, const int32_t *tile, int64_t n, int32_t n_tiles, double *tile_max,
                          int64_t *tile_arg, void *stream) {
    if (n < 0 || n_tiles < 1 || !tile_max || !tile_arg) return TFSC_ERR_ARG;
    if (n > 0 && (!stat || !tile)) return TFSC_ERR_ARG;
    return hip_status(tfsc::launch_tile_max(stat, tile, n, n_tiles, tile_max, tile_arg,
                                            reinterpret_cast<hipStream_t>(stream)));
}

}  // extern "C"

namespace {

// Shared by tfsc_transform (psd_tf NULL: S_m(f_k) = mu_m S0(f_k)) and tfsc_transform_tf (psd_tf set).
tfsc_status transform_common(const tfsc_grid *grid, const void *x, int x_dtype, const double *psd0,
                             const double *mu, const double *psd_tf, const uint8_t *tranche_keep, tfsc_pixels *out,
                             void *ws, size_t ws_bytes, void *stream) {
    if (x_dtype != TFSC_F64 && x_dtype != TFSC_F32) return TFSC_ERR_DTYPE;
    if (out->dtype == TFSC_F64 && x_dtype != TFSC_F64) return TFSC_ERR_DTYPE;
    if (out->dtype == TFSC_F64 && grid->tranche_len > 2048) return TFSC_ERR_UNSUPPORTED;
    const bool q16 = is_16bit(out->dtype);
    if (q16 && (!ws || ws_bytes < ws_bytes_for(grid, 0, TFSC_WS_TRANSFORM))) return TFSC_ERR_WORKSPACE;
    tfsc::TransformLaunch L;
    L.M = grid->tranche_len;
    L.Nt = grid->n_tranches;
    L.C = grid->n_channels;
    L.dt = grid->dt;
    L.alpha = grid->tukey_alpha;
    L.x = x;
    L.x_dtype = x_dtype;
    L.psd0 = psd0;
    L.mu = mu;
    L.psd_tf = psd_tf;
    L.keep = tranche_keep;
    L.out_dtype = out->dtype;
    L.out_layout = out->layout;
    L.pix = out->pix;
    L.layer_scale = out->layer_scale;
    L.inv_asd = out->inv_asd;
    L.tranche_w = out->tranche_w;
    L.rho = psd_tf ? out->rho : nullptr;
    L.ws = ws;
    return hip_status(tfsc::launch_transform(L, reinterpret_cast<hipStream_t>(stream)));
}

}  // namespace

extern "C" {

tfsc_status tfsc_transform(const tfsc_grid *grid, const void *x, int x_dtype, const double *psd0,
                           const double *tranche_psd_scale, const uint8_t *tranche_keep, tfsc_pixels *out,
                           void *ws, size_t ws_bytes, void *stream) {
    tfsc_status s;
    if ((s = check_grid(grid)) != TFSC_OK) return s;
    if ((s = check_pixels(out, true)) != TFSC_OK) return s;
    if (!x || !psd0 || !tranche_psd_scale || !tranche_keep) return TFSC_ERR_ARG;
    return transform_common(grid, x, x_dtype, psd0, tranche_psd_scale, nullptr, tranche_keep, out, ws, ws_bytes,
                            stream);
}

tfsc_status tfsc_transform_tf(const tfsc_grid *grid, const void *x, int x_dtype, const double *psd_tf,
                              const uint8_t *tranche_keep, tfsc_pixels *out, void *ws, size_t ws_bytes,
                              void *stream) {
    tfsc_status s;
    if ((s = check_grid(grid)) != TFSC_OK) return s;
    if ((s = check_pixels(out, true)) != TFSC_OK) return s;
    if (!x || !psd_tf || !tranche_keep || !out->rho) return TFSC_ERR_ARG;
    return transform_common(grid, x, x_dtype, nullptr, nullptr, psd_tf, tranche_keep, out, ws, ws_bytes, stream);
}

tfsc_status tfsc_track(const tfsc_grid *grid, const tfsc_bank *bank, double *out, void *stream) {
    tfsc_status s;
    if ((s = check_grid(grid)) != TFSC_OK) return s;
    if ((s = check_bank(bank)) != TFSC_OK) return s;
    if (bank->n > 0 && !out) return TFSC_ERR_ARG;
    return hip_status(tfsc::launch_track(bank->n, grid->tranche_len, grid->n_tranches, grid->dt, bank->mc,
                                         bank->ln_mc, bank->eta, bank->f0, bank->cos_theta, bank->cos_iota, out,
                                         reinterpret_cast<hipStream_t>(stream)));
}

tfsc_status tfsc_orbit_positions(const tfsc_grid *grid, double *out, void *stream) {
    tfsc_status s;
    if ((s = check_grid(grid)) != TFSC_OK) return s;
    if (!out) return TFSC_ERR_ARG;
    return hip_status(tfsc::launch_orbit_positions(grid->n_tranches, (double)grid->tranche_len * grid->dt, out,
                                                   reinterpret_cast<hipStream_t>(stream)));
}

tfsc_status tfsc_link_lengths(const tfsc_grid *grid, const double *orbit, double *out, void *stream) {
    tfsc_status s;
    if ((s = check_grid(grid)) != TFSC_OK) return s;
    if (!out) return TFSC_ERR_ARG;
    return hip_status(tfsc::launch_link_lengths(grid->n_tranches, (double)grid->tranche_len * grid->dt, orbit, out,
                                                reinterpret_cast<hipStream_t>(stream)));
}

tfsc_status tfsc_bank_statistic_harmonics(const tfsc_grid *grid, const tfsc_pixels *pix, const tfsc_bank *bank,
                                          const tfsc_segments *seg, const tfsc_options *opt, int32_t n_harm,
                                          const int32_t *harmonics, const double *amp, double *seg_terms,
                                          double *stat, double *seg_zn, int32_t *flags, int32_t *n_active, void *ws,
                                          size_t ws_bytes, void *stream) {
    tfsc_status s;
    if ((s = check_grid(grid)) != TFSC_OK) return s;
    if ((s = check_bank(bank)) != TFSC_OK) return s;
    if ((s = check_pixels(pix, bank->n > 0)) != TFSC_OK) return s;
    if (!seg || (bank->n > 0 && (!seg->nseg || !seg->seg_offset))) return TFSC_ERR_ARG;
    if (n_harm < 1 || n_harm > TFSC_MAX_HARMONICS || !harmonics) return TFSC_ERR_ARG;
    for (int q = 0; q < n_harm; ++q) {
        if (harmonics[q] < 1 || harmonics[q] > 8) return TFSC_ERR_ARG;
        for (int r2 = 0; r2 < q; ++r2)
            if (harmonics[r2] == harmonics[q]) return TFSC_ERR_ARG;
    }
    Resolved r;
    if ((s = resolve_options(opt, pix, r)) != TFSC_OK) return s;
    if (r.schedule != TFSC_SCHED_WAVE || r.fresnel != TFSC_FRESNEL_PAPER || pix->rho || pix->links)
        return TFSC_ERR_UNSUPPORTED;
    if (!((pix->dtype == TFSC_F64 && r.precision == TFSC_F64) || (pix->dtype == TFSC_F32 && r.precision == TFSC_F32)))
        return TFSC_ERR_DTYPE;
    if (bank->n > 0 && (!seg_terms || !stat || !flags || !amp)) return TFSC_ERR_ARG;
    if (!ws || ws_bytes < stat_ws_bytes(grid, bank->n, bank->ln_mc != nullptr)) return TFSC_ERR_WORKSPACE;
    if (pixel_store_bytes(grid, pix) > 0xffffffffull) return TFSC_ERR_UNSUPPORTED;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (bank->n == 0) return TFSC_OK;
    tfsc::StatLaunch L = stat_launch(grid, pix, bank, seg, r, ws);
    if (prepare_launch(grid, pix, L, ws, st) != hipSuccess) return TFSC_ERR_HIP;
    L.seg_terms = seg_terms;
    L.stat = stat;
    L.seg_zn = seg_zn;
    L.flags = flags;
    L.n_active = n_active;
    int h[TFSC_MAX_HARMONICS];
    for (int q = 0; q < n_harm; ++q) h[q] = harmonics[q];
    return hip_status(tfsc::launch_statistic_harmonics(L, n_harm, h, amp, st));
}

tfsc_status tfsc_tune_statistic(const tfsc_grid *grid, const tfsc_pixels *pix, const tfsc_bank *bank,
                                const tfsc_segments *seg, const tfsc_options *opt, const char *tune_key,
                                double *seg_terms, double *stat, int32_t *flags, void *ws, size_t ws_bytes,
                                void *stream, int32_t *block_waves, int32_t *groups_per_cu) {
    static const int kCand[][2] = {{4, 4}, {4, 3}, {4, 2}, {2, 8}, {2, 6}, {2, 4}, {1, 12}, {1, 8}};
    if (!tune_key || !block_waves || !groups_per_cu) return TFSC_ERR_ARG;
    tfsc_options o;
    memset(&o, 0, sizeof(o));
    if (opt) o = *opt;
    o.schedule = TFSC_SCHED_WAVE;
    o.tune_key = nullptr;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return TFSC_ERR_HIP;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return TFSC_ERR_HIP;
    }
    // warm-up launch, with the full argument checks
    tfsc_status s = tfsc_bank_statistic(grid, pix, bank, seg, &o, seg_terms, stat, nullptr, flags, nullptr, ws,
                                        ws_bytes, stream);
    float best = 0.0f;
    int bw = 0, gpc = 0;
    for (size_t c = 0; s == TFSC_OK && c < sizeof(kCand) / sizeof(kCand[0]); ++c) {
        o.block_waves = kCand[c][0];
        o.groups_per_cu = kCand[c][1];
        float t = 0.0f;
        for (int rep = 0; rep < 2 && s == TFSC_OK; ++rep) {
            if (hipEventRecord(e0, st) != hipSuccess) s = TFSC_ERR_HIP;
            if (s == TFSC_OK)
                s = tfsc_bank_statistic(grid, pix, bank, seg, &o, seg_terms, stat, nullptr, flags, nullptr, ws,
                                        ws_bytes, stream);
            if (s == TFSC_OK && (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess))
                s = TFSC_ERR_HIP;
            float ms = 0.0f;
            if (s == TFSC_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) s = TFSC_ERR_HIP;
            if (s == TFSC_OK && (rep == 0 || ms < t)) t = ms;
        }
        if (s == TFSC_OK && (bw == 0 || t < best)) {
            best = t;
            bw = kCand[c][0];
            gpc = kCand[c][1];
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (s != TFSC_OK) return s;
    {
        TuneTable &t = tune_table();
        std::lock_guard<std::mutex> lock(t.mu);
        t.shape[tune_key] = std::make_pair(bw, gpc);
    }
    *block_waves = bw;
    *groups_per_cu = gpc;
    return TFSC_OK;
}

}  // extern "C"
