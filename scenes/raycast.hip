// Depth maps of a piecewise-constant heightfield (scene input generation).
//
// The heightfield covers the unit square with N x N cells; cell (i, j)
// spans [i/N, (i+1)/N) x [j/N, (j+1)/N) and has height H[j * N + i].  Each
// pixel ray is walked cell by cell (2-D DDA) from where it enters the box
// [0,1]^2 x [zmin, zmax]; the first cell whose column it meets gives the hit
// (a wall where the ray enters the cell below the top, else the top face).
// Output: camera-frame z of the hit, 0 where the ray leaves the box.
// Arithmetic in float64.  This is input synthesis only.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

struct RayCam {
    double R[9], t[3];
    double fx, fy, cx, cy;
};

__global__ void k_raycast(const float *__restrict__ H, int N, double zmin, double zmax, const RayCam *cams, int W,
                          int Hh, float *__restrict__ out) {
    int px = blockIdx.x * blockDim.x + threadIdx.x;
    int py = blockIdx.y * blockDim.y + threadIdx.y;
    int c = blockIdx.z;
    if (px >= W || py >= Hh) return;
    const RayCam &cm = cams[c];
    double C[3], d[3];
    for (int k = 0; k < 3; k++) C[k] = -(cm.R[k] * cm.t[0] + cm.R[3 + k] * cm.t[1] + cm.R[6 + k] * cm.t[2]);
    double a = (px + 0.5 - cm.cx) / cm.fx, b = (py + 0.5 - cm.cy) / cm.fy;
    for (int k = 0; k < 3; k++) d[k] = cm.R[k] * a + cm.R[3 + k] * b + cm.R[6 + k];
    // slab entry/exit of the box
    double lo[3] = {0.0, 0.0, zmin}, hi[3] = {1.0, 1.0, zmax};
    double t0 = 1e-9, t1 = 1e30;
    bool miss = false;
    for (int k = 0; k < 3; k++) {
        if (fabs(d[k]) < 1e-300) {
            if (C[k] < lo[k] || C[k] > hi[k]) miss = true;
        } else {
            double ta = (lo[k] - C[k]) / d[k], tb = (hi[k] - C[k]) / d[k];
            if (ta > tb) { double tmp = ta; ta = tb; tb = tmp; }
            t0 = fmax(t0, ta);
            t1 = fmin(t1, tb);
        }
    }
    long long o = ((long long)c * Hh + py) * W + px;
    if (miss || t0 >= t1) {
        out[o] = 0.0f;
        return;
    }
    double x = C[0] + t0 * d[0], y = C[1] + t0 * d[1];
    int ci = (int)floor(x * N), cj = (int)floor(y * N);
    ci = ci < 0 ? 0 : (ci > N - 1 ? N - 1 : ci);
    cj = cj < 0 ? 0 : (cj > N - 1 ? N - 1 : cj);
    int si = d[0] > 0 ? 1 : -1, sj = d[1] > 0 ? 1 : -1;
    double tdx = fabs(d[0]) > 1e-300 ? 1.0 / (N * fabs(d[0])) : 1e300;
    double tdy = fabs(d[1]) > 1e-300 ? 1.0 / (N * fabs(d[1])) : 1e300;
    double tmx = fabs(d[0]) > 1e-300 ? ((ci + (si > 0 ? 1 : 0)) / (double)N - C[0]) / d[0] : 1e300;
    double tmy = fabs(d[1]) > 1e-300 ? ((cj + (sj > 0 ? 1 : 0)) / (double)N - C[1]) / d[1] : 1e300;
    double tc = t0;
    float res = 0.0f;
    for (int guard = 0; guard < 4 * N + 8; guard++) {
        double te = fmin(fmin(tmx, tmy), t1);
        double h = H[(long long)cj * N + ci];
        double zin = C[2] + tc * d[2], zout = C[2] + te * d[2];
        if (fmin(zin, zout) <= h) {
            double th = zin <= h ? tc : (h - C[2]) / d[2];
            res = (float)th;
            break;
        }
        if (te >= t1) break;
        tc = te;
        if (tmx < tmy) {
            ci += si;
            tmx += tdx;
        } else {
            cj += sj;
            tmy += tdy;
        }
        if (ci < 0 || cj < 0 || ci >= N || cj >= N) break;
    }
    out[o] = res;
}

extern "C" int scenes_raycast(const float *H_dev, int N, double zmin, double zmax, const double *cams_host, int ncam,
                              int W, int Hh, float *out_dev, void *stream) {
    RayCam *dc = nullptr;
    if (hipMalloc((void **)&dc, sizeof(RayCam) * ncam) != hipSuccess) return 2;
    if (hipMemcpy(dc, cams_host, sizeof(RayCam) * ncam, hipMemcpyHostToDevice) != hipSuccess) return 3;
    dim3 blk(64, 4, 1), grd((W + 63) / 64, (Hh + 3) / 4, ncam);
    hipLaunchKernelGGL(k_raycast, grd, blk, 0, (hipStream_t)stream, H_dev, N, zmin, zmax, dc, W, Hh, out_dev);
    hipError_t e = hipStreamSynchronize((hipStream_t)stream);
    (void)hipFree(dc);
    return e == hipSuccess ? 0 : 4;
}
