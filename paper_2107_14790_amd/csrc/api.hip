// C ABI of libtgv: argument checking, camera culling, workspace and state
// management, and the launch sequence of a solve.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "context.h"

using namespace tgv;

namespace {

tgv_status fail(tgv_ctx *ctx, tgv_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    if (ctx) ctx->err = buf;
    return st;
}

#define HIP_TRY(ctx, call)                                                                           \
    do {                                                                                             \
        hipError_t e_ = (call);                                                                      \
        if (e_ != hipSuccess)                                                                        \
            return fail(ctx, e_ == hipErrorOutOfMemory ? TGV_E_NOMEM : TGV_E_DEVICE, "%s: %s", #call, \
                        hipGetErrorString(e_));                                                      \
    } while (0)

tgv_status check_launch(tgv_ctx *ctx, const char *what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(ctx, TGV_E_DEVICE, "%s launch: %s", what, hipGetErrorString(e));
    return TGV_OK;
}

bool grid_ok(const tgv_grid *g) {
    if (!g) return false;
    if (g->nx < 1 || g->ny < 1 || g->nz < 1 || g->halo < 0) return false;
    int m = std::min(g->nx, std::min(g->ny, g->nz));
    if (2LL * g->halo >= m) return false;
    if (!(g->h > 0.0f) || !isfinite(g->h)) return false;
    for (int i = 0; i < 3; i++)
        if (!isfinite(g->origin[i])) return false;
    long long n = (long long)g->nx * g->ny * g->nz;
    return n <= (1LL << 31) / 8;  // q offsets (6 n) stay far inside 32-bit element counts
}

bool bins_ok(const tgv_bins *b) {
    if (!b || b->num_bins < 1 || b->num_bins > 8) return false;
    if (b->rule != 0 && b->rule != 1) return false;
    if (!(b->delta > 0.0f) || !isfinite(b->delta)) return false;
    if (!(b->eta_over_delta >= 0.0f) || !isfinite(b->eta_over_delta)) return false;
    for (int k = 0; k < b->num_bins; k++) {
        if (!isfinite(b->centers[k])) return false;
        if (k > 0 && !(b->centers[k] > b->centers[k - 1])) return false;
    }
    return true;
}

bool params_ok(const tgv_params *p) {
    if (!p) return false;
    if (!(p->tau > 0.0f) || !(p->sigma > 0.0f) || !isfinite(p->tau) || !isfinite(p->sigma)) return false;
    if (!(p->alpha0 >= 0.0f) || !(p->alpha1 >= 0.0f) || !(p->lambda >= 0.0f)) return false;
    if (!isfinite(p->alpha0) || !isfinite(p->alpha1) || !isfinite(p->lambda)) return false;
    if (p->iters < 0) return false;
    if (p->storage < 0 || p->storage > 2) return false;
    if (p->schedule < TGV_SCHED_FUSED || p->schedule > TGV_SCHED_AUTO) return false;
    if (p->tile_y < 0 || p->tile_z < 0) return false;
    if (p->flags & ~(TGV_FLAG_GRAPH | TGV_FLAG_TVL1 | TGV_FLAG_LEAVE_OPEN)) return false;
    if (p->tile_y != 0) {
        const int cz = p->tile_z > 0 ? p->tile_z : 1;
        if (p->schedule == TGV_SCHED_FUSED2 ? !tiled2_shape_ok(p->tile_y, cz) : !tiled_shape_ok(p->tile_y, cz))
            return false;
    }
    return true;
}

Dims make_dims(const tgv_grid &g) {
    Dims d;
    d.nx = g.nx;
    d.ny = g.ny;
    d.nz = g.nz;
    d.halo = g.halo;
    d.sy = g.nx;
    d.sz = (long long)g.nx * g.ny;
    d.n = d.sz * g.nz;
    return d;
}

Coef make_coef(const tgv_params &p, const tgv_bins &b) {
    Coef c;
    c.alpha0 = p.alpha0;
    c.alpha1 = p.alpha1;
    c.tau = p.tau;
    c.sigma = p.sigma;
    c.taulam = p.tau * p.lambda;
    c.taulam2 = 2.0f * c.taulam;
    for (int k = 0; k < 8; k++) c.c[k] = k < b.num_bins ? b.centers[k] : INFINITY;
    c.tvl1 = (p.flags & TGV_FLAG_TVL1) ? 1 : 0;
    return c;
}

long long align256(long long x) { return (x + 255) & ~255LL; }

SolveBufs bufs_of(const tgv_state *st, int xc, int yc, const uint16_t *hist) {
    SolveBufs b;
    b.xc_u = st->u[xc];
    b.xc_v = st->v[xc];
    b.xo_u = st->u[xc ^ 1];
    b.xo_v = st->v[xc ^ 1];
    b.yc_p = st->p[yc];
    b.yc_q = st->q[yc];
    b.yo_p = st->p[yc ^ 1];
    b.yo_q = st->q[yc ^ 1];
    b.hist = hist;
    return b;
}

hipStream_t S(void *s) { return (hipStream_t)s; }

}  // namespace

// the fixed workspace of tgv_solve_noalloc and its per-device addresses
constexpr int TGV_MAX_DEVICES = 64;
static __device__ __align__(256) unsigned char scratch[TGV_NOALLOC_MAX_BYTES];

static std::mutex g_scratch_mu;
static void *g_scratch_ptr[TGV_MAX_DEVICES];

// the device address of `scratch` on the current device `device`
static tgv_status scratch_lookup(int device) {
    if (device < 0 || device >= TGV_MAX_DEVICES) return TGV_E_DEVICE;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[device]) return TGV_OK;
    void *ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
        (void)hipGetLastError();
        return TGV_E_DEVICE;
    }
    g_scratch_ptr[device] = ptr;
    return TGV_OK;
}

static void *scratch_of(int device) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return (device >= 0 && device < TGV_MAX_DEVICES) ? g_scratch_ptr[device] : nullptr;
}

// ===========================================================================
// context
// ===========================================================================
extern "C" tgv_status tgv_create(int device, tgv_ctx **out) {
    if (!out) return TGV_E_INVAL;
    *out = nullptr;
    if (hipSetDevice(device) != hipSuccess) return TGV_E_DEVICE;
    tgv_ctx *c = new tgv_ctx();
    c->device = device;
    c->cus = 256;
    (void)hipDeviceGetAttribute(&c->cus, hipDeviceAttributeMultiprocessorCount, device);
    c->cams_host = nullptr;
    c->cams_dev = nullptr;
    c->cams_cap = 0;
    c->partials = nullptr;
    c->partials_cap = 0;
    c->eout_dev = nullptr;
    c->eout_host = nullptr;
    c->own = nullptr;
    c->bt_blocks_dev = nullptr;
    c->bt_tiles_dev = nullptr;
    c->bt_blocks_host = nullptr;
    c->bt_tiles_host = nullptr;
    c->bt_blocks_cap = 0;
    c->bt_tiles_cap = 0;
    c->counters = nullptr;
    c->graph_exec = nullptr;
    c->graph_key.clear();
    c->side = nullptr;
    c->ext_scratch = nullptr;
    c->ext_cap = 0;
    c->ext_total_host = nullptr;
    c->c2f_mem = nullptr;
    c->c2f_cap = 0;
    if (hipHostMalloc((void **)&c->ext_total_host, sizeof(unsigned long long), hipHostMallocDefault) != hipSuccess ||
        hipEventCreateWithFlags(&c->cams_evt, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->cams_done, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->own_done, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->c2f_done, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->bt_evt, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->bt_done, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_a, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_b, hipEventDisableTiming) != hipSuccess ||
        hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) != hipSuccess ||
        hipMalloc((void **)&c->counters, 64 * sizeof(int)) != hipSuccess ||
        hipMalloc((void **)&c->eout_dev, sizeof(EnergyOut)) != hipSuccess ||
        hipHostMalloc((void **)&c->eout_host, sizeof(EnergyOut), hipHostMallocDefault) != hipSuccess) {
        delete c;
        return TGV_E_DEVICE;
    }
    if (scratch_lookup(device) != TGV_OK) {
        tgv_destroy(c);
        return TGV_E_DEVICE;
    }
    *out = c;
    return TGV_OK;
}

extern "C" void tgv_destroy(tgv_ctx *c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    if (c->own) tgv_state_destroy(c->own);
    (void)hipFree(c->cams_dev);
    (void)hipHostFree(c->cams_host);
    (void)hipFree(c->partials);
    (void)hipFree(c->eout_dev);
    (void)hipHostFree(c->eout_host);
    (void)hipEventDestroy(c->cams_evt);
    (void)hipEventDestroy(c->cams_done);
    (void)hipEventDestroy(c->own_done);
    (void)hipEventDestroy(c->c2f_done);
    (void)hipEventDestroy(c->bt_evt);
    (void)hipEventDestroy(c->bt_done);
    (void)hipEventDestroy(c->ev_a);
    (void)hipEventDestroy(c->ev_b);
    if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
    (void)hipStreamDestroy(c->side);
    (void)hipFree(c->counters);
    (void)hipFree(c->bt_blocks_dev);
    (void)hipFree(c->bt_tiles_dev);
    (void)hipHostFree(c->bt_blocks_host);
    (void)hipHostFree(c->bt_tiles_host);
    (void)hipFree(c->ext_scratch);
    (void)hipFree(c->c2f_mem);
    (void)hipHostFree(c->ext_total_host);
    delete c;
}

extern "C" const char *tgv_last_error(const tgv_ctx *c) { return c ? c->err.c_str() : "null context"; }

// ===========================================================================
// pyramids
// ===========================================================================
extern "C" int32_t tgv_pyramid_levels(int32_t W, int32_t H) {
    if (W < 1 || H < 1) return 0;
    return pyr_geom(W, H).L;
}

extern "C" int64_t tgv_pyramid_floats(int32_t W, int32_t H) {
    if (W < 1 || H < 1) return 0;
    return pyr_geom(W, H).cam_stride;
}

extern "C" tgv_status tgv_build_pyramids(tgv_ctx *ctx, const float *depth, int32_t n_cams, int32_t W, int32_t H,
                                         float *pyr, void *stream) {
    if (!ctx) return TGV_E_INVAL;
    if (!depth || !pyr || n_cams < 1 || W < 1 || H < 1 || n_cams > 65535)
        return fail(ctx, TGV_E_INVAL, "tgv_build_pyramids: bad arguments");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    PyrGeom g = pyr_geom(W, H);
    if (g.L > 24) return fail(ctx, TGV_E_INVAL, "tgv_build_pyramids: image too large");
    launch_pyramids(depth, n_cams, g, pyr, S(stream));
    return check_launch(ctx, "pyramids");
}

// ===========================================================================
// camera cull and histograms
// ===========================================================================
extern "C" int32_t tgv_cull_cameras(const tgv_camera *cams, int32_t n_cams, const tgv_grid *grid, int32_t *keep) {
    if (!cams || !keep || n_cams < 0 || !grid_ok(grid)) return -1;
    // bounding box of the voxel centres
    double lo[3], hi[3];
    int nn[3] = {grid->nx, grid->ny, grid->nz};
    for (int i = 0; i < 3; i++) {
        lo[i] = (double)grid->origin[i] + 0.5 * grid->h;
        hi[i] = (double)grid->origin[i] + (nn[i] - 0.5) * (double)grid->h;
    }
    int cnt = 0;
    for (int c = 0; c < n_cams; c++) {
        const tgv_camera &cm = cams[c];
        if (cm.model != TGV_MODEL_PINHOLE) {  // a 360-degree scan sees every direction
            keep[cnt++] = c;
            continue;
        }
        double zmin = INFINITY, pxmin = INFINITY, pxmax = -INFINITY, pymin = INFINITY, pymax = -INFINITY;
        bool all_front = true;
        for (int k = 0; k < 8; k++) {
            double P[3] = {(k & 1) ? hi[0] : lo[0], (k & 2) ? hi[1] : lo[1], (k & 4) ? hi[2] : lo[2]};
            double xc[3];
            for (int r = 0; r < 3; r++)
                xc[r] = cm.R[3 * r] * P[0] + cm.R[3 * r + 1] * P[1] + cm.R[3 * r + 2] * P[2] + cm.t[r];
            zmin = std::min(zmin, xc[2]);
            if (xc[2] <= 0.0) {
                all_front = false;
                continue;
            }
            double px = cm.fx * (xc[0] / xc[2]) + cm.cx, py = cm.fy * (xc[1] / xc[2]) + cm.cy;
            pxmin = std::min(pxmin, px);
            pxmax = std::max(pxmax, px);
            pymin = std::min(pymin, py);
            pymax = std::max(pymax, py);
        }
        double zmax_all = -INFINITY;
        for (int k = 0; k < 8; k++) {
            double P[3] = {(k & 1) ? hi[0] : lo[0], (k & 2) ? hi[1] : lo[1], (k & 4) ? hi[2] : lo[2]};
            double z = cm.R[6] * P[0] + cm.R[7] * P[1] + cm.R[8] * P[2] + cm.t[2];
            zmax_all = std::max(zmax_all, z);
        }
        // every voxel centre is a convex combination of the corners: if all
        // corners are behind the camera (with a float32 rounding margin), so
        // is every centre
        double zscale = 1e-5 * (fabs(cm.t[2]) + fabs(hi[0]) + fabs(hi[1]) + fabs(hi[2]) + fabs(lo[0]) + fabs(lo[1]) +
                                fabs(lo[2]) + 1.0);
        if (zmax_all < -zscale) continue;
        if (all_front && zmin > zscale) {
            // projections of centres lie in the convex hull of the corner
            // projections; keep a 2-pixel (+ relative) margin for rounding
            double mx = 2.0 + 1e-5 * (fabs(pxmin) + fabs(pxmax));
            double my = 2.0 + 1e-5 * (fabs(pymin) + fabs(pymax));
            if (pxmax < -mx || pxmin > cm.width + mx || pymax < -my || pymin > cm.height + my) continue;
        }
        keep[cnt++] = c;
    }
    return cnt;
}

// Histograms of `grid` from n_cams cameras, camera c's pyramid at pyr +
// offs[c] floats (each at the camera's own size), the counts added to
// hist's when `accumulate` (whose voxels hold at most `prior` votes).
static tgv_status histograms_impl(tgv_ctx *ctx, const char *who, const float *pyr, const int64_t *offs,
                                  const tgv_camera *cams_host, int32_t n_cams, const tgv_grid *grid,
                                  const tgv_bins *bins, bool accumulate, int32_t prior, uint16_t *hist,
                                  void *stream) {
    if (!pyr || !hist || !cams_host || n_cams < 0 || prior < 0 || (!accumulate && prior != 0))
        return fail(ctx, TGV_E_INVAL, "%s: bad arguments", who);
    if (!grid_ok(grid)) return fail(ctx, TGV_E_INVAL, "%s: bad grid", who);
    if (!bins_ok(bins)) return fail(ctx, TGV_E_INVAL, "%s: bad bins", who);
    for (int c = 0; c < n_cams; c++) {
        const tgv_camera &cm = cams_host[c];
        if (cm.width < 1 || cm.height < 1) return fail(ctx, TGV_E_INVAL, "%s: camera %d is %dx%d", who, c, cm.width, cm.height);
        if (cm.vote < 0 || cm.vote > 65535) return fail(ctx, TGV_E_INVAL, "%s: camera %d has vote %d", who, c, cm.vote);
        if (cm.model != TGV_MODEL_PINHOLE && cm.model != TGV_MODEL_SCAN360)
            return fail(ctx, TGV_E_INVAL, "%s: camera %d has model %d", who, c, cm.model);
        if (cm.model == TGV_MODEL_SCAN360 && (cm.width % 4 != 0 || !(cm.fx > 0.0f) || !isfinite(cm.fx)))
            return fail(ctx, TGV_E_INVAL, "%s: scan %d needs a width divisible by 4 and fx > 0", who, c);
        const PyrGeom g = pyr_geom(cm.width, cm.height);
        if (g.L > 24 || g.cam_stride >= (1LL << 31))
            return fail(ctx, TGV_E_INVAL, "%s: camera %d's image is too large", who, c);
        if (offs[c] < 0) return fail(ctx, TGV_E_INVAL, "%s: camera %d's pyramid offset is negative", who, c);
    }
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    std::vector<int32_t> keep(n_cams > 0 ? n_cams : 1);
    int nk = tgv_cull_cameras(cams_host, n_cams, grid, keep.data());
    long long total = prior;
    for (int k = 0; k < nk; k++) total += cams_host[keep[k]].vote;
    if (total > 65535)
        return fail(ctx, TGV_E_OVERFLOW, "%s: %d votes already possible plus those of %d cameras sum to %lld > 65535",
                    who, prior, nk, total);
    // boundary tables of the kept scans, one set per distinct size
    std::vector<std::pair<long long, int>> tab_of;  // (W << 32 | H, float offset)
    std::vector<int> cam_tab(nk, 0);
    long long tab_floats = 0;
    for (int k = 0; k < nk; k++) {
        const tgv_camera &c = cams_host[keep[k]];
        if (c.model != TGV_MODEL_SCAN360) continue;
        const long long key = ((long long)c.width << 32) | c.height;
        int at = -1;
        for (auto &e : tab_of)
            if (e.first == key) at = e.second;
        if (at < 0) {
            at = (int)tab_floats;
            tab_of.push_back({key, at});
            tab_floats += c.width / 2 + c.height;
        }
        cam_tab[k] = at;
    }
    if (tab_floats >= (1LL << 31)) return fail(ctx, TGV_E_INVAL, "%s: scan tables too large", who);
    // stage the culled camera table and the scan tables (wait until the
    // previous upload left the staging buffer)
    const long long cam_bytes = align256((long long)sizeof(CamDev) * nk);
    const long long need = cam_bytes + 4 * tab_floats;
    HIP_TRY(ctx, hipEventSynchronize(ctx->cams_evt));
    if (need > ctx->cams_cap) {
        const long long cap = std::max(need, (long long)sizeof(CamDev) * 64);
        HIP_TRY(ctx, hipEventSynchronize(ctx->cams_done));  // no kernel reads the old table any more
        (void)hipFree(ctx->cams_dev);
        (void)hipHostFree(ctx->cams_host);
        ctx->cams_dev = nullptr;
        ctx->cams_host = nullptr;
        ctx->cams_cap = 0;
        HIP_TRY(ctx, hipMalloc((void **)&ctx->cams_dev, cap));
        HIP_TRY(ctx, hipHostMalloc((void **)&ctx->cams_host, cap, hipHostMallocDefault));
        ctx->cams_cap = cap;
    }
    CamDev *cd = (CamDev *)ctx->cams_host;
    float *tabs = (float *)(ctx->cams_host + cam_bytes);
    for (auto &e : tab_of) {
        const int W = (int)(e.first >> 32), H = (int)(e.first & 0xffffffff);
        scan_tables(W, H, tabs + e.second, tabs + e.second + W / 4, tabs + e.second + W / 2);
    }
    for (int k = 0; k < nk; k++) {
        const tgv_camera &c = cams_host[keep[k]];
        CamDev &d = cd[k];
        memset(&d, 0, sizeof(d));
        memcpy(d.R, c.R, sizeof(d.R));
        memcpy(d.t, c.t, sizeof(d.t));
        d.fx = c.fx;
        d.fy = c.fy;
        d.cx = c.cx;
        d.cy = c.cy;
        d.vote = c.vote;
        d.model = c.model;
        d.W = c.width;
        d.H = c.height;
        const PyrGeom g = pyr_geom(c.width, c.height);
        d.L = g.L;
        for (int l = 0; l < g.L; l++) d.lvl[l] = (int)g.off[l];
        d.base = offs[keep[k]];
        d.tab = cam_tab[k];
    }
    if (nk > 0) {
        // the previous call's kernel (perhaps on another stream) is done with the table
        HIP_TRY(ctx, hipStreamWaitEvent(S(stream), ctx->cams_done, 0));
        HIP_TRY(ctx, hipMemcpyAsync(ctx->cams_dev, ctx->cams_host, need, hipMemcpyHostToDevice, S(stream)));
        HIP_TRY(ctx, hipEventRecord(ctx->cams_evt, S(stream)));
    }
    launch_histograms(pyr, (const CamDev *)ctx->cams_dev, nk, (const float *)(ctx->cams_dev + cam_bytes), *grid,
                      *bins, accumulate, hist, S(stream));
    tgv_status r = check_launch(ctx, "histograms");
    if (r != TGV_OK) return r;
    HIP_TRY(ctx, hipEventRecord(ctx->cams_done, S(stream)));
    return TGV_OK;
}

extern "C" tgv_status tgv_build_histograms(tgv_ctx *ctx, const float *pyr, int32_t W, int32_t H,
                                           const tgv_camera *cams_host, int32_t n_cams, const tgv_grid *grid,
                                           const tgv_bins *bins, uint16_t *hist, void *stream) {
    if (!ctx) return TGV_E_INVAL;
    if (W < 1 || H < 1 || n_cams < 0 || !cams_host) return fail(ctx, TGV_E_INVAL, "tgv_build_histograms: bad arguments");
    for (int c = 0; c < n_cams; c++)
        if (cams_host[c].width != W || cams_host[c].height != H)
            return fail(ctx, TGV_E_INVAL, "camera %d is %dx%d, pyramids are %dx%d", c, cams_host[c].width,
                        cams_host[c].height, W, H);
    const long long stride = pyr_geom(W, H).cam_stride;
    std::vector<int64_t> offs(n_cams > 0 ? n_cams : 1);
    for (int c = 0; c < n_cams; c++) offs[c] = stride * c;
    return histograms_impl(ctx, "tgv_build_histograms", pyr, offs.data(), cams_host, n_cams, grid, bins, false, 0,
                           hist, stream);
}

extern "C" tgv_status tgv_build_histograms_ex(tgv_ctx *ctx, const float *pyr, const int64_t *pyr_offsets_host,
                                              const tgv_camera *cams_host, int32_t n_cams, const tgv_grid *grid,
                                              const tgv_bins *bins, int32_t flags, int32_t prior_votes,
                                              uint16_t *hist, void *stream) {
    if (!ctx) return TGV_E_INVAL;
    if ((n_cams > 0 && !pyr_offsets_host) || (flags & ~TGV_HIST_ACCUMULATE))
        return fail(ctx, TGV_E_INVAL, "tgv_build_histograms_ex: bad arguments");
    return histograms_impl(ctx, "tgv_build_histograms_ex", pyr, pyr_offsets_host, cams_host, n_cams, grid, bins,
                           (flags & TGV_HIST_ACCUMULATE) != 0, prior_votes, hist, stream);
}

// ===========================================================================
// solver state
// ===========================================================================
extern "C" int64_t tgv_state_bytes(const tgv_grid *grid, int32_t storage) {
    if (!grid_ok(grid) || storage < 0 || storage > 2) return -1;
    long long n = (long long)grid->nx * grid->ny * grid->nz;
    long long sb = storage_bytes(storage);
    return 2 * align256(4 * n) + 2 * align256(3 * n * sb) + 2 * align256(3 * n * sb) + 2 * align256(6 * n * sb);
}

static void state_layout(tgv_state *st) {
    long long sb = storage_bytes(st->storage), n = st->n;
    char *b = (char *)st->mem;
    for (int k = 0; k < 2; k++) {
        st->u[k] = (float *)b;
        b += align256(4 * n);
    }
    for (int k = 0; k < 2; k++) {
        st->v[k] = b;
        b += align256(3 * n * sb);
    }
    for (int k = 0; k < 2; k++) {
        st->p[k] = b;
        b += align256(3 * n * sb);
    }
    for (int k = 0; k < 2; k++) {
        st->q[k] = b;
        b += align256(6 * n * sb);
    }
    st->xc = 0;
    st->yc = 0;
    st->fresh = true;
    st->open = false;
    st->open_tvl1 = 0;
    st->iters_done = 0;
}

extern "C" tgv_status tgv_state_create(tgv_ctx *ctx, const tgv_grid *grid, int32_t storage, tgv_state **out) {
    if (!ctx || !out) return TGV_E_INVAL;
    *out = nullptr;
    if (!grid_ok(grid)) return fail(ctx, TGV_E_INVAL, "tgv_state_create: bad grid");
    if (storage < 0 || storage > 2) return fail(ctx, TGV_E_INVAL, "tgv_state_create: bad storage %d", storage);
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    tgv_state *st = new tgv_state();
    st->grid = *grid;
    st->storage = storage;
    st->n = (long long)grid->nx * grid->ny * grid->nz;
    st->owned = true;
    long long bytes = tgv_state_bytes(grid, storage);
    if (hipMalloc(&st->mem, bytes) != hipSuccess) {
        delete st;
        (void)hipGetLastError();
        return fail(ctx, TGV_E_NOMEM, "tgv_state_create: cannot allocate %lld bytes", bytes);
    }
    state_layout(st);
    *out = st;
    return TGV_OK;
}

extern "C" tgv_status tgv_state_wrap(tgv_ctx *ctx, const tgv_grid *grid, int32_t storage, void *mem, int64_t bytes,
                                     tgv_state **out) {
    if (!ctx || !out) return TGV_E_INVAL;
    *out = nullptr;
    if (!grid_ok(grid)) return fail(ctx, TGV_E_INVAL, "tgv_state_wrap: bad grid");
    if (storage < 0 || storage > 2) return fail(ctx, TGV_E_INVAL, "tgv_state_wrap: bad storage %d", storage);
    if (!mem || ((uintptr_t)mem & 255)) return fail(ctx, TGV_E_INVAL, "tgv_state_wrap: memory not 256-byte aligned");
    if (bytes < tgv_state_bytes(grid, storage))
        return fail(ctx, TGV_E_INVAL, "tgv_state_wrap: %lld bytes < %lld needed", (long long)bytes,
                    (long long)tgv_state_bytes(grid, storage));
    tgv_state *st = new tgv_state();
    st->grid = *grid;
    st->storage = storage;
    st->n = (long long)grid->nx * grid->ny * grid->nz;
    st->owned = false;
    st->mem = mem;
    state_layout(st);
    *out = st;
    return TGV_OK;
}

extern "C" void tgv_state_destroy(tgv_state *st) {
    if (!st) return;
    if (st->owned) (void)hipFree(st->mem);
    delete st;
}

extern "C" tgv_status tgv_state_reset(tgv_ctx *ctx, tgv_state *st, const float *u0, void *stream) {
    if (!ctx) return TGV_E_INVAL;
    if (!st || !u0) return fail(ctx, TGV_E_INVAL, "tgv_state_reset: null argument");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    long long n = st->n, sb = storage_bytes(st->storage);
    st->xc = 0;
    st->yc = 0;
    HIP_TRY(ctx, hipMemcpyAsync(st->u[0], u0, 4 * n, hipMemcpyDeviceToDevice, S(stream)));
    launch_fill_bytes0(st->v[0], 3 * n * sb, S(stream));
    launch_fill_bytes0(st->p[0], 3 * n * sb, S(stream));
    launch_fill_bytes0(st->q[0], 6 * n * sb, S(stream));
    st->fresh = true;
    st->open = false;
    st->iters_done = 0;
    return check_launch(ctx, "state reset");
}

extern "C" tgv_status tgv_state_export(tgv_ctx *ctx, const tgv_state *st, float *u, float *v, float *u_prev,
                                       float *v_prev, float *p, float *q, void *stream) {
    if (!ctx) return TGV_E_INVAL;
    if (!st) return fail(ctx, TGV_E_INVAL, "tgv_state_export: null state");
    if (st->open) return fail(ctx, TGV_E_INVAL, "tgv_state_export: the state is open (close it with a solve)");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    long long n = st->n;
    int xp = st->fresh ? st->xc : (st->xc ^ 1);
    if (u) HIP_TRY(ctx, hipMemcpyAsync(u, st->u[st->xc], 4 * n, hipMemcpyDeviceToDevice, S(stream)));
    if (u_prev) HIP_TRY(ctx, hipMemcpyAsync(u_prev, st->u[xp], 4 * n, hipMemcpyDeviceToDevice, S(stream)));
    if (v) launch_convert(st->v[st->xc], st->storage, v, 0, 3 * n, S(stream));
    if (v_prev) launch_convert(st->v[xp], st->storage, v_prev, 0, 3 * n, S(stream));
    if (p) launch_convert(st->p[st->yc], st->storage, p, 0, 3 * n, S(stream));
    if (q) launch_convert(st->q[st->yc], st->storage, q, 0, 6 * n, S(stream));
    return check_launch(ctx, "state export");
}

extern "C" tgv_status tgv_state_import(tgv_ctx *ctx, tgv_state *st, const float *u, const float *v,
                                       const float *u_prev, const float *v_prev, const float *p, const float *q,
                                       int64_t iters_done, void *stream) {
    if (!ctx) return TGV_E_INVAL;
    if (!st || !u || !v || !u_prev || !v_prev || !p || !q)
        return fail(ctx, TGV_E_INVAL, "tgv_state_import: null argument");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    long long n = st->n;
    st->xc = 0;
    st->yc = 0;
    st->fresh = false;
    st->open = false;
    HIP_TRY(ctx, hipMemcpyAsync(st->u[0], u, 4 * n, hipMemcpyDeviceToDevice, S(stream)));
    HIP_TRY(ctx, hipMemcpyAsync(st->u[1], u_prev, 4 * n, hipMemcpyDeviceToDevice, S(stream)));
    launch_convert(v, 0, st->v[0], st->storage, 3 * n, S(stream));
    launch_convert(v_prev, 0, st->v[1], st->storage, 3 * n, S(stream));
    launch_convert(p, 0, st->p[0], st->storage, 3 * n, S(stream));
    launch_convert(q, 0, st->q[0], st->storage, 6 * n, S(stream));
    st->iters_done = iters_done;
    return check_launch(ctx, "state import");
}

// ===========================================================================
// solve
// ===========================================================================
// TV-L1 (Eq. 1) has no v and no q: both iterates of each are set to 0, so
// every kernel reads and writes zeros there (and the two-iteration kernel
// can leave them alone)
static void zero_vq(tgv_state *st, hipStream_t s) {
    const long long n = st->n, sb = storage_bytes(st->storage);
    for (int k = 0; k < 2; k++) {
        launch_fill_bytes0(st->v[k], 3 * n * sb, s);
        launch_fill_bytes0(st->q[k], 6 * n * sb, s);
    }
}

static bool same_grid(const tgv_grid &a, const tgv_grid &b) {
    return a.nx == b.nx && a.ny == b.ny && a.nz == b.nz && a.halo == b.halo;
}

static tgv_status run_energy(tgv_ctx *ctx, const tgv_state *st, const uint16_t *hist, const tgv_bins *bins,
                             const tgv_params *params, tgv_stats *out, hipStream_t s) {
    if (st->open) return fail(ctx, TGV_E_INVAL, "energy: the state is open (close it with a solve)");
    Dims d = make_dims(st->grid);
    Coef cf = make_coef(*params, *bins);
    int np = energy_partials(d);
    if (np > ctx->partials_cap) {
        (void)hipFree(ctx->partials);
        ctx->partials = nullptr;
        ctx->partials_cap = 0;
        HIP_TRY(ctx, hipMalloc((void **)&ctx->partials, sizeof(double) * 5 * np));
        ctx->partials_cap = np;
    }
    SolveBufs b = bufs_of(st, st->xc, st->yc, hist);
    launch_energy(st->storage, b, d, cf, params->lambda, 2.0 * sqrt(3.0), ctx->partials, np, ctx->eout_dev, s);
    tgv_status r = check_launch(ctx, "energy");
    if (r != TGV_OK) return r;
    HIP_TRY(ctx, hipMemcpyAsync(ctx->eout_host, ctx->eout_dev, sizeof(EnergyOut), hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    const EnergyOut &e = *ctx->eout_host;
    out->parts[0] = e.part[0];
    out->parts[1] = e.part[1];
    out->parts[2] = e.part[2];
    out->primal = e.part[0] + e.part[1] + e.part[2];
    out->dual = e.dual;
    out->gap_rel = (out->primal - out->dual) / std::max(out->primal, 1.0);
    out->nonfinite = (int64_t)e.nonfinite;
    out->iters_done = st->iters_done;
    return TGV_OK;
}

extern "C" tgv_status tgv_energy(tgv_ctx *ctx, const tgv_state *st, const uint16_t *hist, const tgv_bins *bins,
                                 const tgv_params *params, tgv_stats *stats_host, void *stream) {
    if (!ctx) return TGV_E_INVAL;
    if (!st || !hist || !stats_host) return fail(ctx, TGV_E_INVAL, "tgv_energy: null argument");
    if (!bins_ok(bins) || !params_ok(params)) return fail(ctx, TGV_E_INVAL, "tgv_energy: bad bins or params");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    return run_energy(ctx, st, hist, bins, params, stats_host, S(stream));
}

// params->iters iterations on a state (kernels only: nothing is allocated).
// A closed state starts with its opening dual step (the first iteration's
// dual half); each fused pass then completes one iteration's primal half
// and the next one's dual half; the closing primal step completes the last
// iteration unless TGV_FLAG_LEAVE_OPEN keeps the state open for the next
// call, which then starts with a fused pass.
static tgv_status advance(tgv_ctx *ctx, tgv_state *st, const uint16_t *hist, const tgv_bins *bins,
                          const tgv_params *params, hipStream_t s) {
    Dims d = make_dims(st->grid);
    Coef cf = make_coef(*params, *bins);
    const int N = params->iters;
    const bool leave_open = (params->flags & TGV_FLAG_LEAVE_OPEN) != 0;
    if (st->open && cf.tvl1 != st->open_tvl1)
        return fail(ctx, TGV_E_INVAL, "solve: an open state continues with the model it was opened with");
    if (!st->open && N == 0) return TGV_OK;
    int F = N;  // fused passes
    if (!st->open) {
        if (cf.tvl1) zero_vq(st, s);
        // opening dual step from (x^n, x^{n-1}, y^n): y^{n+1}, in place
        SolveBufs b = bufs_of(st, st->xc, st->yc, hist);
        if (st->fresh) {
            b.xo_u = b.xc_u;
            b.xo_v = b.xc_v;
        }
        launch_ref(KIND_DUAL, st->storage, b, d, cf, s);
        st->open = true;
        st->open_tvl1 = cf.tvl1;
        st->fresh = false;
        F = N - 1;
    }
    // AUTO: two iterations per pass unless the block is small (measured
    // crossover near 96^3 in float32 and 16-bit storage: 48 MiB per iteration)
    int sched = params->schedule;
    if (sched == TGV_SCHED_AUTO) {
        const long long per_voxel = st->storage == 0 ? 120 : 72;
        sched = (params->tile_y == 0 && d.n * per_voxel > (48LL << 20)) ? TGV_SCHED_FUSED2 : TGV_SCHED_FUSED;
    }
    if (sched == TGV_SCHED_SPLIT) {
        // a fused pass as its two per-voxel kernels
        for (int it = 0; it < F; it++) {
            launch_ref(KIND_PRIMAL, st->storage, bufs_of(st, st->xc, st->yc, hist), d, cf, s);
            st->xc ^= 1;
            launch_ref(KIND_DUAL, st->storage, bufs_of(st, st->xc, st->yc, hist), d, cf, s);
        }
    } else if (F > 0) {
        int ty = params->tile_y ? params->tile_y : default_tile_y(st->storage, d);
        int cz = params->tile_z ? params->tile_z
                                : choose_tile_z(d, ty, ctx->cus * tiled_blocks_per_cu(st->storage, ty, d));
        int it = 0;
        if (sched == TGV_SCHED_FUSED2 && tiled_fits(d)) {
            // pairs of fused passes in one sweep; x^{n+1} is never written,
            // which only the closing primal pass could notice, and it
            // overwrites that buffer
            const int ty2 = params->tile_y ? params->tile_y : DEFAULT_TILE2_Y;
            const int cz2 = params->tile_z ? params->tile_z
                                           : choose_tile2_z(d, ty2, ctx->cus * tiled2_blocks_per_cu(st->storage, ty2));
            for (; it + 2 <= F; it += 2) {
                launch_tiled2(st->storage, bufs_of(st, st->xc, st->yc, hist), d, cf, ty2, cz2, s);
                st->xc ^= 1;
                st->yc ^= 1;
            }
            ty = default_tile_y(st->storage, d);
            if (!params->tile_z) cz = choose_tile_z(d, ty, ctx->cus * tiled_blocks_per_cu(st->storage, ty, d));
        }
        for (; it < F; it++) {
            SolveBufs b = bufs_of(st, st->xc, st->yc, hist);
            if (sched == TGV_SCHED_FUSED_REF) launch_ref(KIND_FUSED, st->storage, b, d, cf, s);
            else launch_tiled(st->storage, b, d, cf, ty, cz, s);
            st->xc ^= 1;
            st->yc ^= 1;
        }
    }
    if (!leave_open) {
        launch_ref(KIND_PRIMAL, st->storage, bufs_of(st, st->xc, st->yc, hist), d, cf, s);
        st->xc ^= 1;
        st->open = false;
    }
    st->iters_done += N;
    return check_launch(ctx, "solve");
}

extern "C" tgv_status tgv_solve(tgv_ctx *ctx, const tgv_grid *grid, const uint16_t *hist, const tgv_bins *bins,
                                const tgv_params *params, float *u_io, tgv_state *state, tgv_stats *stats_host,
                                void *stream) {
    if (!ctx) return TGV_E_INVAL;
    if (!grid_ok(grid)) return fail(ctx, TGV_E_INVAL, "tgv_solve: bad grid");
    if (!bins_ok(bins)) return fail(ctx, TGV_E_INVAL, "tgv_solve: bad bins");
    if (!params_ok(params)) return fail(ctx, TGV_E_INVAL, "tgv_solve: bad params");
    if (!hist) return fail(ctx, TGV_E_INVAL, "tgv_solve: null hist");
    if (!state && !u_io) return fail(ctx, TGV_E_INVAL, "tgv_solve: fresh solve needs u_io");
    if ((params->flags & TGV_FLAG_LEAVE_OPEN) && (!state || u_io || stats_host))
        return fail(ctx, TGV_E_INVAL, "tgv_solve: TGV_FLAG_LEAVE_OPEN needs a state and no u_io or statistics");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipStream_t s = S(stream);
    tgv_state *st = state;
    if (st) {
        if (!same_grid(st->grid, *grid) || st->storage != params->storage)
            return fail(ctx, TGV_E_INVAL, "tgv_solve: state does not match grid/storage");
    } else {
        if (ctx->own && (!same_grid(ctx->own->grid, *grid) || ctx->own->storage != params->storage)) {
            HIP_TRY(ctx, hipEventSynchronize(ctx->own_done));  // the last solve on it has finished
            tgv_state_destroy(ctx->own);
            ctx->own = nullptr;
        }
        if (!ctx->own) {
            tgv_status r = tgv_state_create(ctx, grid, params->storage, &ctx->own);
            if (r != TGV_OK) return r;
        }
        st = ctx->own;
        st->grid = *grid;
        HIP_TRY(ctx, hipStreamWaitEvent(s, ctx->own_done, 0));  // a solve on another stream may still use it
        tgv_status r = tgv_state_reset(ctx, st, u_io, stream);
        if (r != TGV_OK) return r;
    }
    {
        tgv_status r = advance(ctx, st, hist, bins, params, s);
        if (r != TGV_OK) return r;
    }
    if (u_io) HIP_TRY(ctx, hipMemcpyAsync(u_io, st->u[st->xc], 4 * st->n, hipMemcpyDeviceToDevice, s));
    if (!state) HIP_TRY(ctx, hipEventRecord(ctx->own_done, s));
    if (stats_host) return run_energy(ctx, st, hist, bins, params, stats_host, s);
    return TGV_OK;
}


// A fresh solve (u = u_io, v = p = q = 0, params->iters iterations, u back
// to u_io) on a state laid over `mem` (tgv_state_bytes(grid, storage) bytes,
// 256-byte aligned): kernels and device copies only, nothing allocated.
static tgv_status fresh_solve_on(tgv_ctx *ctx, void *mem, const tgv_grid *grid, const uint16_t *hist,
                                 const tgv_bins *bins, const tgv_params *params, float *u_io, hipStream_t s) {
    if (params->flags & TGV_FLAG_LEAVE_OPEN) return fail(ctx, TGV_E_INVAL, "fresh solve: TGV_FLAG_LEAVE_OPEN");
    tgv_state st{};
    st.grid = *grid;
    st.storage = params->storage;
    st.n = (long long)grid->nx * grid->ny * grid->nz;
    st.owned = false;
    st.mem = mem;
    state_layout(&st);
    // fresh start: u = u_io, v = p = q = 0 (fill kernels, no memset)
    HIP_TRY(ctx, hipMemcpyAsync(st.u[0], u_io, 4 * st.n, hipMemcpyDeviceToDevice, s));
    const long long sb = storage_bytes(st.storage);
    launch_fill_bytes0(st.v[0], 3 * st.n * sb, s);
    launch_fill_bytes0(st.p[0], 3 * st.n * sb, s);
    launch_fill_bytes0(st.q[0], 6 * st.n * sb, s);
    tgv_status r = advance(ctx, &st, hist, bins, params, s);
    if (r != TGV_OK) return r;
    HIP_TRY(ctx, hipMemcpyAsync(u_io, st.u[st.xc], 4 * st.n, hipMemcpyDeviceToDevice, s));
    return check_launch(ctx, "fresh solve");
}

// ---------------------------------------------------------------------------
// Fresh solve without allocation: the solver state lives in `scratch`, a
// fixed array in device memory (one per GPU the library runs on, held until
// the process ends).  Host code never passes the array's name to a kernel or
// a copy: it is a host-side stand-in, not a device address.  tgv_create looks
// up each device's address of the array once, with that device current, and
// every use goes through that pointer.
// ---------------------------------------------------------------------------
extern "C" tgv_status tgv_solve_noalloc(tgv_ctx *ctx, const tgv_grid *grid, const uint16_t *hist,
                                        const tgv_bins *bins, const tgv_params *params, float *u_io, void *stream) {
    if (!ctx) return TGV_E_INVAL;
    if (!grid_ok(grid)) return fail(ctx, TGV_E_INVAL, "tgv_solve_noalloc: bad grid");
    if (!bins_ok(bins)) return fail(ctx, TGV_E_INVAL, "tgv_solve_noalloc: bad bins");
    if (!params_ok(params)) return fail(ctx, TGV_E_INVAL, "tgv_solve_noalloc: bad params");
    if (!hist || !u_io) return fail(ctx, TGV_E_INVAL, "tgv_solve_noalloc: null hist or u_io");
    const long long need = tgv_state_bytes(grid, params->storage);
    if (need < 0 || need > TGV_NOALLOC_MAX_BYTES)
        return fail(ctx, TGV_E_INVAL,
                    "tgv_solve_noalloc: the state of a %d x %d x %d block needs %lld bytes, more than the %lld "
                    "of the fixed workspace",
                    grid->nx, grid->ny, grid->nz, need, (long long)TGV_NOALLOC_MAX_BYTES);
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    void *mem = scratch_of(ctx->device);
    if (!mem) return fail(ctx, TGV_E_DEVICE, "tgv_solve_noalloc: no workspace address for device %d", ctx->device);
    return fresh_solve_on(ctx, mem, grid, hist, bins, params, u_io, S(stream));
}

// ===========================================================================
// batched solve
// ===========================================================================
// Chunk depth of the blocks of a batched two-iteration launch when none is
// given.  A tile of c planes takes c + 3 plane steps (the two stages'
// pipeline fill and the z-halo); the launch lasts about its plane steps per
// resident workgroup plus one tile for the tail.  The depth in {16, 32, 64}
// minimising that is taken (ties: the deeper): many blocks take deep chunks
// (less halo), a few small blocks shallow ones (the chip stays full).  On the
// 512 city blocks this takes 64 planes (2.88 s against 3.01 s with a fixed 32).
static int batch2_chunk(tgv_ctx *ctx, int n, tgv_state *const *states, int storage, int ty) {
    const double slots = (double)ctx->cus * batch2_blocks_per_cu(storage, ty);
    int best = 32;
    double best_cost = 0.0;
    for (int cz : {16, 32, 64}) {
        double steps = 0.0;
        int longest = 0;
        for (int i = 0; i < n; i++) {
            const Dims d = make_dims(states[i]->grid);
            if (!tiled_fits(d)) continue;
            const double cols = (double)((d.nx + 63) / 64) * ((d.ny + ty - 1) / ty);
            steps += cols * (d.nz + 3.0 * ((d.nz + cz - 1) / cz));
            longest = std::max(longest, std::min(cz, d.nz) + 3);
        }
        const double cost = steps / slots + longest;
        if (cz == 16 || cost <= best_cost) {
            best_cost = cost;
            best = cz;
        }
    }
    return best;
}

// chunk depth of a block in a batched launch (bcz: the batch's two-iteration depth)
static int batch_tile_z(const Dims &d, bool two, int bcz) {
    if (!two) return DEFAULT_TILE_Z;
    return d.nz < bcz ? d.nz : bcz;
}

static int persistent_grid(tgv_ctx *ctx, int storage, int ty, int ntiles, bool two) {
    // as many workgroups as can be resident at once (occupancy of the batched kernel)
    int g = ctx->cus * (two ? batch2_blocks_per_cu(storage, ty) : batch_blocks_per_cu(storage, ty));
    g = (g + 7) / 8 * 8;
    int cap = (ntiles + 7) / 8 * 8;
    return g < cap ? g : cap;
}

extern "C" tgv_status tgv_solve_batch(tgv_ctx *ctx, int32_t n, tgv_state *const *states, const uint16_t *const *hist,
                                      const tgv_bins *bins, const tgv_params *params, const int32_t *tile_z_host,
                                      tgv_stats *stats_host, void *stream) {
    if (!ctx) return TGV_E_INVAL;
    if (n < 0 || (n > 0 && (!states || !hist))) return fail(ctx, TGV_E_INVAL, "tgv_solve_batch: bad arguments");
    if (!bins_ok(bins)) return fail(ctx, TGV_E_INVAL, "tgv_solve_batch: bad bins");
    if (!params_ok(params)) return fail(ctx, TGV_E_INVAL, "tgv_solve_batch: bad params");
    for (int i = 0; i < n; i++) {
        if (!states[i] || !hist[i]) return fail(ctx, TGV_E_INVAL, "tgv_solve_batch: null state or hist %d", i);
        if (states[i]->storage != params->storage)
            return fail(ctx, TGV_E_INVAL, "tgv_solve_batch: state %d storage %d != %d", i, states[i]->storage,
                        params->storage);
        if (tile_z_host && tile_z_host[i] < 1) return fail(ctx, TGV_E_INVAL, "tgv_solve_batch: tile_z[%d] < 1", i);
        for (int j = 0; j < i; j++)
            if (states[j] == states[i]) return fail(ctx, TGV_E_INVAL, "tgv_solve_batch: state %d repeated", i);
    }
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipStream_t s = S(stream);
    Coef cf = make_coef(*params, *bins);
    const int N = params->iters;
    // two iterations per launch (FUSED2, or AUTO without a given tile), else one
    const bool two = params->schedule == TGV_SCHED_FUSED2 || (params->schedule == TGV_SCHED_AUTO && params->tile_y == 0);
    const int ty = params->tile_y ? params->tile_y : (two ? DEFAULT_TILE2_Y : DEFAULT_BATCH_TILE_Y);
    if (two ? !tiled2_shape_ok(ty, 1) : !tiled_shape_ok(ty, 1))
        return fail(ctx, TGV_E_INVAL, "tgv_solve_batch: tile_y %d", ty);
    const bool leave_open = (params->flags & TGV_FLAG_LEAVE_OPEN) != 0;
    if (leave_open && stats_host)
        return fail(ctx, TGV_E_INVAL, "tgv_solve_batch: TGV_FLAG_LEAVE_OPEN with statistics");
    for (int i = 0; i < n; i++)
        if (states[i]->open && states[i]->open_tvl1 != cf.tvl1)
            return fail(ctx, TGV_E_INVAL, "tgv_solve_batch: open state %d continues with the model it was opened with", i);
    if (n == 0 || N == 0) {
        // nothing to advance: close the open states unless they stay open
        for (int i = 0; i < n && !leave_open; i++) {
            tgv_state *st = states[i];
            if (!st->open) continue;
            launch_ref(KIND_PRIMAL, st->storage, bufs_of(st, st->xc, st->yc, hist[i]), make_dims(st->grid), cf, s);
            st->xc ^= 1;
            st->open = false;
        }
        tgv_status r = check_launch(ctx, "batched solve");
        if (r != TGV_OK) return r;
        if (stats_host)
            for (int i = 0; i < n; i++) {
                r = run_energy(ctx, states[i], hist[i], bins, params, &stats_host[i], s);
                if (r != TGV_OK) return r;
            }
        return TGV_OK;
    }
    // 1. opening dual step of every closed block (in place).  A block that
    //    came open needs N fused passes, one opened here N - 1: with both
    //    kinds in the batch, the blocks that came open take one extra
    //    batched pass first, over the head of the tile table (they are
    //    listed first)
    std::vector<char> came_open(n, 0);
    bool any_open = false, any_closed = false;
    for (int i = 0; i < n; i++) {
        tgv_state *st = states[i];
        came_open[i] = st->open ? 1 : 0;
        any_open |= st->open;
        any_closed |= !st->open;
        if (st->open) continue;
        if (cf.tvl1) zero_vq(st, s);
        SolveBufs b = bufs_of(st, st->xc, st->yc, hist[i]);
        if (st->fresh) {
            b.xo_u = b.xc_u;
            b.xo_v = b.xc_v;
        }
        launch_ref(KIND_DUAL, st->storage, b, make_dims(st->grid), cf, s);
        st->open = true;
        st->open_tvl1 = cf.tvl1;
        st->fresh = false;
    }
    const bool extra = any_open && any_closed;
    // blocks in table order: those that came open first
    std::vector<int> order;
    for (int pass = 0; pass < 2; pass++)
        for (int i = 0; i < n; i++)
            if ((came_open[i] != 0) == (pass == 0)) order.push_back(i);
    // 2. block and tile tables (blocks too large for 32-bit tile offsets run alone)
    std::vector<int> big;
    HIP_TRY(ctx, hipEventSynchronize(ctx->bt_evt));  // the previous upload has left the staging buffers
    int nb = 0, nt = 0, nt_extra = 0;
    bool all_span = true;
    const int bcz = (two && !tile_z_host && !params->tile_z) ? batch2_chunk(ctx, n, states, params->storage, ty) : 32;
    {
        long long tiles = 0;
        for (int i = 0; i < n; i++) {
            Dims d = make_dims(states[i]->grid);
            if (!tiled_fits(d)) continue;
            int cz = tile_z_host ? tile_z_host[i] : (params->tile_z ? params->tile_z : batch_tile_z(d, two, bcz));
            tiles += (long long)((d.nx + 63) / 64) * ((d.ny + ty - 1) / ty) * ((d.nz + cz - 1) / cz);
        }
        if (tiles > (1LL << 30)) return fail(ctx, TGV_E_INVAL, "tgv_solve_batch: too many tiles");
        // a captured graph holds the table addresses: drop it before a table moves
        if (n > ctx->bt_blocks_cap || tiles > ctx->bt_tiles_cap)
            HIP_TRY(ctx, hipEventSynchronize(ctx->bt_done));  // no launch reads the old tables any more
        if ((n > ctx->bt_blocks_cap || tiles > ctx->bt_tiles_cap) && ctx->graph_exec) {
            HIP_TRY(ctx, hipStreamSynchronize(ctx->side));
            (void)hipGraphExecDestroy(ctx->graph_exec);
            ctx->graph_exec = nullptr;
            ctx->graph_key.clear();
        }
        if (n > ctx->bt_blocks_cap) {
            (void)hipFree(ctx->bt_blocks_dev);
            (void)hipHostFree(ctx->bt_blocks_host);
            ctx->bt_blocks_dev = nullptr;
            ctx->bt_blocks_host = nullptr;
            ctx->bt_blocks_cap = 0;
            HIP_TRY(ctx, hipMalloc((void **)&ctx->bt_blocks_dev, sizeof(BatchBlock) * n));
            HIP_TRY(ctx, hipHostMalloc((void **)&ctx->bt_blocks_host, sizeof(BatchBlock) * n, hipHostMallocDefault));
            ctx->bt_blocks_cap = n;
        }
        if (tiles > ctx->bt_tiles_cap) {
            (void)hipFree(ctx->bt_tiles_dev);
            (void)hipHostFree(ctx->bt_tiles_host);
            ctx->bt_tiles_dev = nullptr;
            ctx->bt_tiles_host = nullptr;
            ctx->bt_tiles_cap = 0;
            HIP_TRY(ctx, hipMalloc((void **)&ctx->bt_tiles_dev, sizeof(int4) * tiles));
            HIP_TRY(ctx, hipHostMalloc((void **)&ctx->bt_tiles_host, sizeof(int4) * tiles, hipHostMallocDefault));
            ctx->bt_tiles_cap = (int)tiles;
        }
        for (int i : order) {
            tgv_state *st = states[i];
            Dims d = make_dims(st->grid);
            if (!tiled_fits(d)) {
                big.push_back(i);
                continue;
            }
            int cz = tile_z_host ? tile_z_host[i] : (params->tile_z ? params->tile_z : batch_tile_z(d, two, bcz));
            BatchBlock &bb = ctx->bt_blocks_host[nb];
            for (int k = 0; k < 2; k++) {
                bb.u[k] = st->u[k];
                bb.v[k] = st->v[k];
                bb.p[k] = st->p[k];
                bb.q[k] = st->q[k];
            }
            bb.hist = hist[i];
            bb.d = d;
            bb.cz = cz;
            // parity seen by the common passes: after the extra pass for a
            // block that came open (which runs with flip 1)
            const int pre = (extra && came_open[i]) ? 1 : 0;
            bb.xc = st->xc ^ pre;
            bb.yc = st->yc ^ pre;
            // state_layout puts every field in one allocation from u[0]
            const long long sbytes = tgv_state_bytes(&st->grid, st->storage);
            bb.span = sbytes < (1LL << 31) ? (int)sbytes : 0;
            all_span = all_span && bb.span > 0;
            int ntx = (d.nx + 63) / 64, nty = (d.ny + ty - 1) / ty, ntz = (d.nz + cz - 1) / cz;
            for (int z = 0; z < ntz; z++)
                for (int y = 0; y < nty; y++)
                    for (int x = 0; x < ntx; x++) ctx->bt_tiles_host[nt++] = make_int4(nb, x | (y << 16), z, 0);
            if (extra && came_open[i]) nt_extra = nt;
            nb++;
        }
    }
    if (nb > 0) {
        // the previous batched solve (perhaps on another stream) is done with the tables and counters
        HIP_TRY(ctx, hipStreamWaitEvent(s, ctx->bt_done, 0));
        HIP_TRY(ctx, hipMemcpyAsync(ctx->bt_blocks_dev, ctx->bt_blocks_host, sizeof(BatchBlock) * nb,
                                    hipMemcpyHostToDevice, s));
        HIP_TRY(ctx, hipMemcpyAsync(ctx->bt_tiles_dev, ctx->bt_tiles_host, sizeof(int4) * nt, hipMemcpyHostToDevice, s));
        HIP_TRY(ctx, hipEventRecord(ctx->bt_evt, s));
    }
    // 3. fused passes of all blocks: N - 1 after an opening dual step, N
    //    when every block came open; first the extra pass of the blocks
    //    that came open in a mixed batch (one-iteration batched launch over
    //    their tiles)
    if (extra && nt_extra > 0) {
        int g1 = ctx->cus * batch_blocks_per_cu(params->storage, ty);
        g1 = (g1 + 7) / 8 * 8;
        const int cap = (nt_extra + 7) / 8 * 8;
        launch_batch(params->storage, ctx->bt_blocks_dev, (const int4 *)ctx->bt_tiles_dev, nt_extra, ctx->counters,
                     cf, ty, 1, g1 < cap ? g1 : cap, s);
    }
    const int grid = persistent_grid(ctx, params->storage, ty, nt, two);
    const int F = any_closed ? N - 1 : N;
    // batched launches: F one-iteration passes, or F/2 two-iteration passes
    // (plus, for an odd F, one one-iteration pass per block after them)
    const int LB = two ? F / 2 : F;
    auto launch_one = [&](int flip, hipStream_t st_) {
        if (two)
            launch_batch2(params->storage, ctx->bt_blocks_dev, (const int4 *)ctx->bt_tiles_dev, nt, ctx->counters, cf,
                          ty, flip, grid, all_span, st_);
        else
            launch_batch(params->storage, ctx->bt_blocks_dev, (const int4 *)ctx->bt_tiles_dev, nt, ctx->counters, cf,
                         ty, flip, grid, st_);
    };
    if (nb > 0 && LB > 0) {
        const bool use_graph = (params->flags & TGV_FLAG_GRAPH) && LB >= 2;
        if (!use_graph) {
            for (int it = 0; it < LB; it++) launch_one(it & 1, s);
        } else {
            // the graph holds two launches (parity 0 then 1); it is keyed by
            // everything its kernel arguments capture
            char key[256];
            int kl = snprintf(key, sizeof(key), "%d|%d|%d|%d|%d|%d|%d|%p|%p|%p|", params->storage, (int)two, ty, nt,
                              grid, nb, (int)all_span, (void *)ctx->bt_blocks_dev, (void *)ctx->bt_tiles_dev,
                              (void *)ctx->counters);
            std::string k(key, kl);
            k.append((const char *)&cf, sizeof(cf));
            HIP_TRY(ctx, hipEventRecord(ctx->ev_a, s));
            HIP_TRY(ctx, hipStreamWaitEvent(ctx->side, ctx->ev_a, 0));
            if (!ctx->graph_exec || ctx->graph_key != k) {
                if (ctx->graph_exec) {
                    HIP_TRY(ctx, hipStreamSynchronize(ctx->side));  // no replay of the old graph in flight
                    (void)hipGraphExecDestroy(ctx->graph_exec);
                    ctx->graph_exec = nullptr;
                }
                hipGraph_t g = nullptr;
                HIP_TRY(ctx, hipStreamBeginCapture(ctx->side, hipStreamCaptureModeThreadLocal));
                for (int it = 0; it < 2; it++) launch_one(it, ctx->side);
                HIP_TRY(ctx, hipStreamEndCapture(ctx->side, &g));
                hipError_t e = hipGraphInstantiate(&ctx->graph_exec, g, nullptr, nullptr, 0);
                (void)hipGraphDestroy(g);
                if (e != hipSuccess) {
                    ctx->graph_exec = nullptr;
                    return fail(ctx, TGV_E_DEVICE, "graph instantiate: %s", hipGetErrorString(e));
                }
                ctx->graph_key = k;
            }
            for (int r = 0; r < LB / 2; r++) HIP_TRY(ctx, hipGraphLaunch(ctx->graph_exec, ctx->side));
            if (LB & 1) launch_one(0, ctx->side);
            HIP_TRY(ctx, hipEventRecord(ctx->ev_b, ctx->side));
            HIP_TRY(ctx, hipStreamWaitEvent(s, ctx->ev_b, 0));
        }
    }
    // the odd pass left by two-iteration launches: one batched one-iteration
    // launch over the same tile table
    const bool leftover = two && (F & 1) && nb > 0;
    if (leftover) {
        int g1 = ctx->cus * batch_blocks_per_cu(params->storage, ty);
        g1 = (g1 + 7) / 8 * 8;
        const int cap = (nt + 7) / 8 * 8;
        launch_batch(params->storage, ctx->bt_blocks_dev, (const int4 *)ctx->bt_tiles_dev, nt, ctx->counters, cf, ty,
                     LB & 1, g1 < cap ? g1 : cap, s);
    }
    if (nb > 0) HIP_TRY(ctx, hipEventRecord(ctx->bt_done, s));
    // buffer flips of a tiled block (one per launch) and of a block too large
    // for the tiled kernels (one per iteration)
    const int tiled_flips = LB + (leftover ? 1 : 0);
    // blocks too large for the batched kernel: their own fused launches
    for (int i : big) {
        tgv_state *st = states[i];
        Dims d = make_dims(st->grid);
        int xc = st->xc, yc = st->yc;
        const int Fi = F + ((extra && came_open[i]) ? 1 : 0);
        for (int it = 0; it < Fi; it++) {
            launch_ref(KIND_FUSED, st->storage, bufs_of(st, xc, yc, hist[i]), d, cf, s);
            xc ^= 1;
            yc ^= 1;
        }
    }
    // 4. parities after the fused passes, then the closing primal step
    //    unless the states stay open
    for (int i = 0; i < n; i++) {
        tgv_state *st = states[i];
        const int flips = (tiled_fits(make_dims(st->grid)) ? tiled_flips : F) + ((extra && came_open[i]) ? 1 : 0);
        st->xc ^= (flips & 1);
        st->yc ^= (flips & 1);
        if (!leave_open) {
            launch_ref(KIND_PRIMAL, st->storage, bufs_of(st, st->xc, st->yc, hist[i]), make_dims(st->grid), cf, s);
            st->xc ^= 1;
            st->open = false;
        }
        st->iters_done += N;
    }
    tgv_status r = check_launch(ctx, "batched solve");
    if (r != TGV_OK) return r;
    if (stats_host)
        for (int i = 0; i < n; i++) {
            r = run_energy(ctx, states[i], hist[i], bins, params, &stats_host[i], s);
            if (r != TGV_OK) return r;
        }
    return TGV_OK;
}


// ===========================================================================
// zero-level crossings
// ===========================================================================
extern "C" tgv_status tgv_extract_crossings(tgv_ctx *ctx, const tgv_grid *grid, const float *u, float *points,
                                            int64_t max_points, int64_t *count_host, void *stream) {
    if (!ctx) return TGV_E_INVAL;
    if (!grid_ok(grid)) return fail(ctx, TGV_E_INVAL, "tgv_extract_crossings: bad grid");
    if (!u || !count_host || max_points < 0 || (max_points > 0 && !points))
        return fail(ctx, TGV_E_INVAL, "tgv_extract_crossings: bad arguments");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipStream_t s = S(stream);
    Dims d = make_dims(*grid);
    long long nb = extract_blocks(d), nr = extract_runs(d);
    long long need = align256(4 * nb) + align256(8 * (nb + 1)) + 8 * nr;
    if (need > ctx->ext_cap) {
        HIP_TRY(ctx, hipStreamSynchronize(s));
        (void)hipFree(ctx->ext_scratch);
        ctx->ext_scratch = nullptr;
        ctx->ext_cap = 0;
        HIP_TRY(ctx, hipMalloc(&ctx->ext_scratch, need));
        ctx->ext_cap = need;
    }
    unsigned *counts = (unsigned *)ctx->ext_scratch;
    unsigned long long *offsets = (unsigned long long *)((char *)ctx->ext_scratch + align256(4 * nb));
    unsigned long long *runs = (unsigned long long *)((char *)offsets + align256(8 * (nb + 1)));
    launch_extract(u, d, *grid, counts, offsets, runs, (float4 *)points, max_points, s);
    tgv_status r = check_launch(ctx, "extract crossings");
    if (r != TGV_OK) return r;
    HIP_TRY(ctx, hipMemcpyAsync(ctx->ext_total_host, offsets + nb, sizeof(unsigned long long), hipMemcpyDeviceToHost,
                                s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    *count_host = (int64_t)*ctx->ext_total_host;
    return TGV_OK;
}


// ===========================================================================
// coarse-to-fine
// ===========================================================================
extern "C" tgv_status tgv_prolongate(tgv_ctx *ctx, const tgv_grid *coarse, const float *u_coarse, const tgv_grid *fine,
                                     float *u_fine, void *stream) {
    if (!ctx) return TGV_E_INVAL;
    if (!grid_ok(coarse) || !grid_ok(fine) || !u_coarse || !u_fine)
        return fail(ctx, TGV_E_INVAL, "tgv_prolongate: bad arguments");
    if (coarse->nx != (fine->nx + 1) / 2 || coarse->ny != (fine->ny + 1) / 2 || coarse->nz != (fine->nz + 1) / 2)
        return fail(ctx, TGV_E_INVAL, "tgv_prolongate: coarse grid must be ceil(n/2) per axis");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    launch_prolongate(u_coarse, make_dims(*coarse), u_fine, make_dims(*fine), S(stream));
    return check_launch(ctx, "prolongate");
}

extern "C" tgv_status tgv_solve_coarse_to_fine(tgv_ctx *ctx, const float *pyr, int32_t W, int32_t H,
                                               const tgv_camera *cams_host, int32_t n_cams, const tgv_grid *grid,
                                               const tgv_bins *bins, const tgv_params *params, int32_t levels,
                                               float *u_out, void *stream) {
    if (!ctx) return TGV_E_INVAL;
    if (!grid_ok(grid) || !bins_ok(bins) || !params_ok(params) || !u_out || levels < 1 || levels > 16)
        return fail(ctx, TGV_E_INVAL, "tgv_solve_coarse_to_fine: bad arguments");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipStream_t s = S(stream);
    std::vector<tgv_grid> g(levels);
    g[0] = *grid;
    for (int k = 1; k < levels; k++) {
        g[k] = g[k - 1];
        g[k].h = g[k - 1].h * 2.0f;
        g[k].nx = (g[k - 1].nx + 1) / 2;
        g[k].ny = (g[k - 1].ny + 1) / 2;
        g[k].nz = (g[k - 1].nz + 1) / 2;
        g[k].halo = 0;
    }
    // workspace: every level's histograms and u, then one solver state of
    // the finest (largest) level that each level's solve lays itself over
    std::vector<long long> off_h(levels), off_u(levels);
    long long need = 0;
    for (int k = 0; k < levels; k++) {
        const long long n = (long long)g[k].nx * g[k].ny * g[k].nz;
        off_h[k] = need;
        need += align256(16 * n);
        off_u[k] = need;
        need += align256(4 * n);
    }
    const long long off_state = need;
    need += tgv_state_bytes(&g[0], params->storage);
    if (need > ctx->c2f_cap) {
        HIP_TRY(ctx, hipEventSynchronize(ctx->c2f_done));  // the last call's work on it has finished
        (void)hipFree(ctx->c2f_mem);
        ctx->c2f_mem = nullptr;
        ctx->c2f_cap = 0;
        if (hipMalloc(&ctx->c2f_mem, need) != hipSuccess) {
            (void)hipGetLastError();
            return fail(ctx, TGV_E_NOMEM, "tgv_solve_coarse_to_fine: cannot allocate %lld bytes", need);
        }
        ctx->c2f_cap = need;
    }
    HIP_TRY(ctx, hipStreamWaitEvent(s, ctx->c2f_done, 0));  // a call on another stream may still use it
    char *ws = (char *)ctx->c2f_mem;
    tgv_status r = TGV_OK;
    for (int k = levels - 1; k >= 0 && r == TGV_OK; k--) {
        tgv_bins bk = *bins;
        bk.delta = bins->delta * (float)(1 << k);
        uint16_t *hk = (uint16_t *)(ws + off_h[k]);
        float *uk = (float *)(ws + off_u[k]);
        r = tgv_build_histograms(ctx, pyr, W, H, cams_host, n_cams, &g[k], &bk, hk, stream);
        if (r != TGV_OK) break;
        const long long n = (long long)g[k].nx * g[k].ny * g[k].nz;
        if (k == levels - 1) launch_fill(uk, 0.0f, n, s);
        else launch_prolongate((const float *)(ws + off_u[k + 1]), make_dims(g[k + 1]), uk, make_dims(g[k]), s);
        r = fresh_solve_on(ctx, ws + off_state, &g[k], hk, &bk, params, uk, s);
    }
    if (r == TGV_OK) {
        hipError_t e = hipMemcpyAsync(u_out, ws + off_u[0], 4LL * g[0].nx * g[0].ny * g[0].nz,
                                      hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) r = fail(ctx, TGV_E_DEVICE, "copy: %s", hipGetErrorString(e));
    }
    HIP_TRY(ctx, hipEventRecord(ctx->c2f_done, s));
    return r;
}


// ===========================================================================
// streaming copy (measurement)
// ===========================================================================
extern "C" tgv_status tgv_stream_copy(tgv_ctx *ctx, const void *src, void *dst, int64_t bytes, int32_t variant,
                                      void *stream) {
    if (!ctx) return TGV_E_INVAL;
    if (!src || !dst || bytes < 0 || (bytes & 15) || ((uintptr_t)src & 15) || ((uintptr_t)dst & 15) ||
        !stream_copy_variant_ok(variant))
        return fail(ctx, TGV_E_INVAL, "tgv_stream_copy: bad arguments");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    if (bytes == 0) return TGV_OK;
    launch_stream_copy(src, dst, bytes / 16, variant, ctx->cus, S(stream));
    return check_launch(ctx, "stream copy");
}
