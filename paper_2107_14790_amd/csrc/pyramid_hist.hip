// Depth-map mipmap pyramids and voxel-centric vote histograms (Sec. 3.4,
// Algorithm 1).  Canonical binary32: this file is compiled without FMA
// contraction and with correctly rounded division, so every rounding step
// is the one the rule states and integer counts are exact.
#include "internal.h"

namespace tgv {

PyrGeom pyr_geom(int W, int H) {
    PyrGeom g{};
    g.W = W;
    g.H = H;
    long long off = 0;
    int w = W, h = H, l = 0;
    while (true) {
        g.off[l] = off;
        g.w[l] = w;
        g.h[l] = h;
        off += (long long)w * h;
        l++;
        if (w == 1 && h == 1) break;
        w = (w + 1) >> 1;
        h = (h + 1) >> 1;
    }
    g.L = l;
    g.cam_stride = off;
    return g;
}

// level 0: input with invalid samples (not finite or <= 0) set to 0
__global__ void k_pyr_level0(const float *__restrict__ depth, float *__restrict__ pyr, int W, int H,
                             long long cam_stride) {
    int x = blockIdx.x * blockDim.x + threadIdx.x;
    int y = blockIdx.y * blockDim.y + threadIdx.y;
    int c = blockIdx.z;
    if (x >= W || y >= H) return;
    float d = depth[(long long)c * W * H + (long long)y * W + x];
    pyr[(long long)c * cam_stride + (long long)y * W + x] = (isfinite(d) && d > 0.0f) ? d : 0.0f;
}

// level l+1 pixel = mean of the valid children, summed in the order
// (2i,2j), (2i+1,2j), (2i,2j+1), (2i+1,2j+1)
__global__ void k_pyr_down(float *__restrict__ pyr, long long src_off, long long dst_off, int w, int h, int w2,
                           int h2, long long cam_stride) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int j = blockIdx.y * blockDim.y + threadIdx.y;
    int c = blockIdx.z;
    if (i >= w2 || j >= h2) return;
    const float *src = pyr + (long long)c * cam_stride + src_off;
    float sum = 0.0f;
    int cnt = 0;
#pragma unroll
    for (int k = 0; k < 4; k++) {
        int cx = 2 * i + (k & 1), cy = 2 * j + (k >> 1);
        if (cx < w && cy < h) {
            float d = src[(long long)cy * w + cx];
            if (d > 0.0f) {
                sum = sum + d;
                cnt++;
            }
        }
    }
    pyr[(long long)c * cam_stride + dst_off + (long long)j * w2 + i] = cnt ? sum / (float)cnt : 0.0f;
}

void launch_pyramids(const float *depth, int ncam, const PyrGeom &g, float *pyr, hipStream_t s) {
    dim3 blk(64, 4, 1);
    hipLaunchKernelGGL(k_pyr_level0, dim3((g.W + 63) / 64, (g.H + 3) / 4, ncam), blk, 0, s, depth, pyr, g.W, g.H,
                       g.cam_stride);
    for (int l = 0; l + 1 < g.L; l++) {
        int w2 = g.w[l + 1], h2 = g.h[l + 1];
        hipLaunchKernelGGL(k_pyr_down, dim3((w2 + 63) / 64, (h2 + 3) / 4, ncam), blk, 0, s, pyr, g.off[l],
                           g.off[l + 1], g.w[l], g.h[l], w2, h2, g.cam_stride);
    }
}

// Boundary tables of an equirectangular W x H scan (host; W a multiple of
// 4): C[i] = cos(2 pi i / W), S[i] = sin(2 pi i / W) for i < W/4 (one
// quadrant's column boundaries), K[j] = cos(pi j / H) for j < H (row
// boundaries), each evaluated in double and rounded to float.
void scan_tables(int W, int H, float *C, float *S, float *K) {
    for (int i = 0; i < W / 4; i++) {
        const double a = (6.283185307179586 * (double)i) / (double)W;
        C[i] = (float)cos(a);
        S[i] = (float)sin(a);
    }
    for (int j = 0; j < H; j++) {
        const double a = (3.141592653589793 * (double)j) / (double)H;
        K[j] = (float)cos(a);
    }
}

// Column of scanner-frame direction (x, y) in an equirectangular map of W
// columns: turn it by a multiple of -90 degrees into the first quadrant
// (exact), then count the quadrant's boundaries at or before it,
//   #{i in [1, W/4) : C[i] y' - S[i] x' >= 0}  (each product rounded).
// The count is monotone in i (C falls, S rises, x', y' >= 0), so it is
// found by walking from an atan2 estimate to where the test changes: a few
// table reads instead of W/4, and the same integer as counting them all.
__device__ __forceinline__ int scan_column(float x, float y, int W, const float *__restrict__ C,
                                           const float *__restrict__ S) {
    int q;
    float xp, yp;
    if (x > 0.0f && y >= 0.0f) { q = 0; xp = x; yp = y; }
    else if (x <= 0.0f && y > 0.0f) { q = 1; xp = y; yp = -x; }
    else if (x < 0.0f && y <= 0.0f) { q = 2; xp = -x; yp = -y; }
    else if (x >= 0.0f && y < 0.0f) { q = 3; xp = -y; yp = x; }
    else { q = 0; xp = x; yp = y; }
    const int Q = W >> 2;
    int c;
    if (xp == 0.0f && yp == 0.0f) {
        c = Q - 1;  // on the scanner's axis every test reads 0 >= 0
    } else {
        const float est = atan2f(yp, xp) * ((float)W * 0.159154943f);
        c = est > 0.0f ? (int)est : 0;
        c = c < Q - 1 ? c : Q - 1;
        auto at_or_before = [&](int i) { return C[i] * yp - S[i] * xp >= 0.0f; };
        while (c + 1 < Q && at_or_before(c + 1)) c++;
        while (c > 0 && !at_or_before(c)) c--;
    }
    return q * Q + c;
}

// Row of direction z (of length rho) in an equirectangular map of H rows:
// #{j in [1, H) : z <= K[j] rho}, monotone in j, walked from an acos estimate.
__device__ __forceinline__ int scan_row(float z, float rho, int H, const float *__restrict__ K) {
    const float ct = fminf(1.0f, fmaxf(-1.0f, z * __builtin_amdgcn_rcpf(rho)));
    const float est = acosf(ct) * ((float)H * 0.318309886f);
    int r = est > 0.0f ? (int)est : 0;
    r = r < H - 1 ? r : H - 1;
    while (r + 1 < H && z <= K[r + 1] * rho) r++;
    while (r > 0 && !(z <= K[r] * rho)) r--;
    return r;
}

// One thread per voxel; the camera loop is uniform, so camera parameters
// come through scalar loads.  Counts live in two 64-bit registers as four
// 16-bit fields each (the host rules out carries between fields).
__global__ void __launch_bounds__(256) k_hist(const float *__restrict__ pyr, const CamDev *__restrict__ cams, int ncam,
                                              const float *__restrict__ tables, tgv_grid grid, int nbins, int rule,
                                              float delta, float eta, int accumulate, uint16_t *__restrict__ hist) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int j = blockIdx.y * blockDim.y + threadIdx.y;
    int k = blockIdx.z;
    if (i >= grid.nx || j >= grid.ny) return;
    const float h = grid.h;
    const float X = grid.origin[0] + ((float)i + 0.5f) * h;
    const float Y = grid.origin[1] + ((float)j + 0.5f) * h;
    const float Z = grid.origin[2] + ((float)k + 0.5f) * h;
    const float half = (float)(nbins - 1) / 2.0f;
    const float nbf = (float)nbins;
    const long long idx = (long long)i + (long long)grid.nx * (j + (long long)grid.ny * k);
    uint64_t lo = 0, hi = 0;
    if (accumulate) {
        const uint4 w = *reinterpret_cast<const uint4 *>(hist + 8 * idx);
        lo = (uint64_t)w.x | ((uint64_t)w.y << 32);
        hi = (uint64_t)w.z | ((uint64_t)w.w << 32);
    }
    for (int c = 0; c < ncam; c++) {
        const CamDev &cm = cams[c];
        float xc[3];
#pragma unroll
        for (int r = 0; r < 3; r++) {
            float acc = cm.R[3 * r + 0] * X;
            acc = acc + cm.R[3 * r + 1] * Y;
            acc = acc + cm.R[3 * r + 2] * Z;
            xc[r] = acc + cm.t[r];
        }
        float dist, px, py;
        if (cm.model == TGV_MODEL_PINHOLE) {
            const float z = xc[2];
            if (!(z > 0.0f)) continue;
            px = cm.fx * (xc[0] / z) + cm.cx;
            py = cm.fy * (xc[1] / z) + cm.cy;
            if (!(px >= 0.0f && px < (float)cm.W && py >= 0.0f && py < (float)cm.H)) continue;
            dist = z;
        } else {
            float r2 = xc[0] * xc[0];
            r2 = r2 + xc[1] * xc[1];
            r2 = r2 + xc[2] * xc[2];
            const float rho = sqrtf(r2);
            if (!(rho > 0.0f)) continue;
            const float *tb = tables + cm.tab;
            px = (float)scan_column(xc[0], xc[1], cm.W, tb, tb + (cm.W >> 2));
            py = (float)scan_row(xc[2], rho, cm.H, tb + (cm.W >> 1));
            dist = rho;
        }
        float s = (h * cm.fx) / dist;
        int l = 0;
        if (s >= 1.0f) {
            l = ilogbf(s);
            if (l > cm.L - 1) l = cm.L - 1;
        }
        const int wl = ((cm.W - 1) >> l) + 1, hl = ((cm.H - 1) >> l) + 1;
        int ix = (int)floorf(ldexpf(px, -l));
        int iy = (int)floorf(ldexpf(py, -l));
        ix = ix > wl - 1 ? wl - 1 : ix;
        iy = iy > hl - 1 ? hl - 1 : iy;
        float dep = pyr[cm.base + cm.lvl[l] + (long long)iy * wl + ix];
        if (dep == 0.0f) continue;
        float a = dep - dist;
        if (a < -eta) continue;
        float an = fminf(1.0f, fmaxf(-1.0f, a / delta));
        int bin;
        if (rule == 0) bin = (int)floorf((an + 1.0f) * half + 0.5f);
        else bin = (int)floorf(((an + 1.0f) / 2.0f) * nbf);
        bin = bin < 0 ? 0 : (bin > nbins - 1 ? nbins - 1 : bin);
        uint64_t add = (uint64_t)(uint32_t)cm.vote << (16 * (bin & 3));
        if (bin < 4) lo += add;
        else hi += add;
    }
    uint4 w;
    w.x = (uint32_t)lo;
    w.y = (uint32_t)(lo >> 32);
    w.z = (uint32_t)hi;
    w.w = (uint32_t)(hi >> 32);
    *reinterpret_cast<uint4 *>(hist + 8 * idx) = w;
}

void launch_histograms(const float *pyr, const CamDev *cams, int ncam, const float *tables, const tgv_grid &grid,
                       const tgv_bins &bins, bool accumulate, uint16_t *hist, hipStream_t s) {
    float eta = bins.eta_over_delta * bins.delta;
    dim3 blk(64, 4, 1);
    hipLaunchKernelGGL(k_hist, dim3((grid.nx + 63) / 64, (grid.ny + 3) / 4, grid.nz), blk, 0, s, pyr, cams, ncam,
                       tables, grid, bins.num_bins, bins.rule, bins.delta, eta, accumulate ? 1 : 0, hist);
}

// ---------------------------------------------------------------------------
// small utility kernels (graph-capture safe replacements for memset/copies)
// ---------------------------------------------------------------------------
__global__ void k_fill(float *p, float v, long long n) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_fill0_u32(uint32_t *p, long long n) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        p[i] = 0u;
}

static int fill_blocks(long long n) {
    long long b = (n + 255) / 256;
    return (int)(b > 8192 ? 8192 : (b < 1 ? 1 : b));
}

void launch_fill(float *p, float v, long long n, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill, dim3(fill_blocks(n)), dim3(256), 0, s, p, v, n);
}

// Zero nbytes rounded up to whole 32-bit words: a 16-bit field array of an
// odd voxel count ends on a half word, and its last element must be cleared
// too.  Every caller's array is padded to 256 bytes, so the rounding stays
// inside the allocation.
void launch_fill_bytes0(void *p, long long nbytes, hipStream_t s) {
    long long n = (nbytes + 3) / 4;
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill0_u32, dim3(fill_blocks(n)), dim3(256), 0, s, (uint32_t *)p, n);
}

template <int SS, int DS>
__global__ void k_convert(const typename Store<SS>::T *src, typename Store<DS>::T *dst, long long n) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        Store<DS>::st(dst + i, Store<SS>::ld(src + i));
}

template <int SS>
static void convert_to(const void *src, void *dst, int ds, long long n, hipStream_t s) {
    const typename Store<SS>::T *sp = (const typename Store<SS>::T *)src;
    if (ds == 0) hipLaunchKernelGGL((k_convert<SS, 0>), dim3(fill_blocks(n)), dim3(256), 0, s, sp, (float *)dst, n);
    else if (ds == 1)
        hipLaunchKernelGGL((k_convert<SS, 1>), dim3(fill_blocks(n)), dim3(256), 0, s, sp, (__half *)dst, n);
    else hipLaunchKernelGGL((k_convert<SS, 2>), dim3(fill_blocks(n)), dim3(256), 0, s, sp, (bf16_t *)dst, n);
}

void launch_convert(const void *src, int ss, void *dst, int ds, long long n, hipStream_t s) {
    if (n <= 0) return;
    if (ss == 0) convert_to<0>(src, dst, ds, n, s);
    else if (ss == 1) convert_to<1>(src, dst, ds, n, s);
    else convert_to<2>(src, dst, ds, n, s);
}

int64_t storage_bytes(int storage) { return storage == 0 ? 4 : 2; }

}  // namespace tgv
