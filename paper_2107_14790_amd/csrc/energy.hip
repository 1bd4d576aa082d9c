// Energy and duality-gap reduction of a solver state in float64 (the only
// float64 arithmetic on the GPU).  Per voxel: the three terms of Eq. 2 at
// (u, v) and the dual bound of the box-restricted problem at (p, q); the
// block sums are reduced with wavefront shuffles, then the block partials
// in a fixed order by one workgroup, so the result is deterministic.
#include "fields.h"
#include "internal.h"

namespace tgv {

constexpr int EN_THREADS = 256;
constexpr int EN_MAX_BLOCKS = 2048;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ double data_term(double w, const float h[8], const Coef &cf) {
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < 8; k++)
        if (h[k] != 0.0f) s += (double)h[k] * fabs(w - (double)cf.c[k]);
    return s;
}

// four waves per SIMD (at most 128 VGPRs, no spill): at the compiler's own
// choice (254 VGPRs, two waves) the kernel waited on its loads, 1461 against
// 895 us on a 256^3 block
template <int STORE>
__global__ void __launch_bounds__(EN_THREADS, 4) k_energy(XBuf<STORE> X, YBuf<STORE> Y, const uint16_t *hist, Dims d,
                                                       Coef cf, double lambda, double vbound, double *partials) {
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    const double a0 = cf.alpha0, a1 = cf.alpha1;
    for (long long idx = (long long)blockIdx.x * EN_THREADS + threadIdx.x; idx < d.n;
         idx += (long long)gridDim.x * EN_THREADS) {
        // coordinates in 32-bit arithmetic (a block holds at most 2^28
        // voxels): two 32-bit divisions instead of three 64-bit ones
        const unsigned i32 = (unsigned)idx, row = i32 / (unsigned)d.nx, zq = row / (unsigned)d.ny;
        const int x = (int)(i32 - row * (unsigned)d.nx);
        const int y = (int)(row - zq * (unsigned)d.ny);
        const int z = (int)zq;
        Pos s = make_pos(d, x, y, z);
        bool frozen = is_frozen(d, x, y, z);
        double u = X.u[idx];
        double v[3], p[3], q[6];
        for (int c = 0; c < 3; c++) v[c] = Store<STORE>::ld(X.v + c * d.n + idx);
        for (int c = 0; c < 3; c++) p[c] = Store<STORE>::ld(Y.p + c * d.n + idx);
        for (int c = 0; c < 6; c++) q[c] = Store<STORE>::ld(Y.q + c * d.n + idx);
        bool fin = isfinite(u);
        for (int c = 0; c < 3; c++) fin = fin && isfinite(v[c]) && isfinite(p[c]);
        for (int c = 0; c < 6; c++) fin = fin && isfinite(q[c]);
        // primal: alpha1 |M.(grad u - v)|, alpha0 |E v|, data
        double kp2 = 0.0;
        for (int i = 0; i < 3; i++) {
            if (s.mhi[i]) {
                double g = ((double)X.u[idx + axis_stride(d, i)] - u) - v[i];
                kp2 += g * g;
            }
        }
        double dm[3][3];
        for (int i = 0; i < 3; i++)
            for (int j = 0; j < 3; j++)
                dm[i][j] = s.mlo[j] ? v[i] - (double)Store<STORE>::ld(X.v + i * d.n + idx - axis_stride(d, j)) : 0.0;
        double e3 = 0.5 * (dm[0][1] + dm[1][0]), e4 = 0.5 * (dm[0][2] + dm[2][0]), e5 = 0.5 * (dm[1][2] + dm[2][1]);
        double eq2 = dm[0][0] * dm[0][0] + dm[1][1] * dm[1][1] + dm[2][2] * dm[2][2] +
                     2.0 * (e3 * e3 + e4 * e4 + e5 * e5);
        uint32_t hw[4];
        load_hist(hist, idx, hw);
        float h[8];
        for (int k = 0; k < 4; k++) {
            h[2 * k] = (float)(hw[k] & 0xffffu);
            h[2 * k + 1] = (float)(hw[k] >> 16);
        }
        acc[0] += a1 * sqrt(kp2);
        acc[1] += a0 * sqrt(eq2);
        if (!frozen) acc[2] += lambda * data_term(u, h, cf);
        // dual: (gu, gv) = K^T(p, q)
        double gu = 0.0;
        for (int i = 0; i < 3; i++) {
            if (s.mhi[i]) gu -= p[i];
            if (s.mlo[i]) gu += (double)Store<STORE>::ld(Y.p + i * d.n + idx - axis_stride(d, i));
        }
        double gv2 = 0.0;
        for (int i = 0; i < 3; i++) {
            double g = s.mhi[i] ? -p[i] : 0.0;
            for (int j = 0; j < 3; j++) {
                int sl = qslot(i, j);
                if (s.mlo[j]) g += q[sl];
                if (s.mhi[j]) g -= (double)Store<STORE>::ld(Y.q + sl * d.n + idx + axis_stride(d, j));
            }
            gv2 += g * g;
        }
        double dv;
        if (frozen) {
            dv = u * gu;
        } else {
            dv = -1.0 * gu + lambda * data_term(-1.0, h, cf);
            double t = gu + lambda * data_term(1.0, h, cf);
            dv = t < dv ? t : dv;
            for (int k = 0; k < 8; k++) {
                double c = cf.c[k];
                if (c >= -1.0 && c <= 1.0) {
                    double t2 = c * gu + lambda * data_term(c, h, cf);
                    dv = t2 < dv ? t2 : dv;
                }
            }
        }
        acc[3] += cf.tvl1 ? dv : dv - vbound * sqrt(gv2);
        acc[4] += fin ? 0.0 : 1.0;
    }
    __shared__ double sh[EN_THREADS / 64][5];
    int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int k = 0; k < 5; k++) {
        double w = wave_sum(acc[k]);
        if (lane == 0) sh[wv][k] = w;
    }
    __syncthreads();
    if (threadIdx.x < 5) {
        double t = 0.0;
        for (int w = 0; w < EN_THREADS / 64; w++) t += sh[w][threadIdx.x];
        partials[(long long)blockIdx.x * 5 + threadIdx.x] = t;
    }
}

__global__ void __launch_bounds__(EN_THREADS) k_energy_final(const double *partials, int nparts, EnergyOut *out) {
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < nparts; b += EN_THREADS)
        for (int k = 0; k < 5; k++) acc[k] += partials[(long long)b * 5 + k];
    __shared__ double sh[EN_THREADS / 64][5];
    int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int k = 0; k < 5; k++) {
        double w = wave_sum(acc[k]);
        if (lane == 0) sh[wv][k] = w;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double t[5];
        for (int k = 0; k < 5; k++) {
            t[k] = 0.0;
            for (int w = 0; w < EN_THREADS / 64; w++) t[k] += sh[w][k];
        }
        out->part[0] = t[0];
        out->part[1] = t[1];
        out->part[2] = t[2];
        out->dual = t[3];
        out->nonfinite = t[4];
    }
}

int energy_partials(const Dims &d) {
    long long b = (d.n + EN_THREADS - 1) / EN_THREADS;
    return (int)(b < EN_MAX_BLOCKS ? (b < 1 ? 1 : b) : EN_MAX_BLOCKS);
}

template <int STORE>
static void launch_energy_t(const SolveBufs &b, const Dims &d, const Coef &cf, float lambda, double vbound,
                            double *partials, int nparts, EnergyOut *out, hipStream_t s) {
    XBuf<STORE> X{b.xc_u, (typename Store<STORE>::T *)b.xc_v};
    YBuf<STORE> Y{(typename Store<STORE>::T *)b.yc_p, (typename Store<STORE>::T *)b.yc_q};
    hipLaunchKernelGGL(k_energy<STORE>, dim3(nparts), dim3(EN_THREADS), 0, s, X, Y, b.hist, d, cf, (double)lambda,
                       vbound, partials);
    hipLaunchKernelGGL(k_energy_final, dim3(1), dim3(EN_THREADS), 0, s, partials, nparts, out);
}

void launch_energy(int storage, const SolveBufs &b, const Dims &d, const Coef &cf, float lambda, double vbound,
                   double *partials, int nparts, EnergyOut *out, hipStream_t s) {
    if (storage == 0) launch_energy_t<0>(b, d, cf, lambda, vbound, partials, nparts, out, s);
    else if (storage == 1) launch_energy_t<1>(b, d, cf, lambda, vbound, partials, nparts, out, s);
    else launch_energy_t<2>(b, d, cf, lambda, vbound, partials, nparts, out, s);
}

}  // namespace tgv
