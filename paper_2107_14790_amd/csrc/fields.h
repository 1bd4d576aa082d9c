// Solver state fields in device memory and the per-voxel gathers the solver
// kernels share.
#pragma once

#include "device_math.h"

namespace tgv {

// One primal iterate: u (float32) and v (3 components, component-major).
template <int STORE>
struct XBuf {
    float *u;
    typename Store<STORE>::T *v;
};

// One dual iterate: p (3 components) and q (6 components, xx yy zz xy xz yz).
template <int STORE>
struct YBuf {
    typename Store<STORE>::T *p;
    typename Store<STORE>::T *q;
};

template <int STORE>
__device__ __forceinline__ float rnd(float v) {
    typename Store<STORE>::T t;
    Store<STORE>::st(&t, v);
    return Store<STORE>::ld(&t);
}

struct Pos {
    int x, y, z;
    long long idx;
    bool mlo[3], mhi[3];  // x_i > 0, x_i < n_i - 1
};

__device__ __forceinline__ Pos make_pos(const Dims &d, int x, int y, int z) {
    Pos s;
    s.x = x;
    s.y = y;
    s.z = z;
    s.idx = (long long)x + d.sy * y + d.sz * z;
    s.mlo[0] = x > 0;
    s.mlo[1] = y > 0;
    s.mlo[2] = z > 0;
    s.mhi[0] = x < d.nx - 1;
    s.mhi[1] = y < d.ny - 1;
    s.mhi[2] = z < d.nz - 1;
    return s;
}

__device__ __forceinline__ long long axis_stride(const Dims &d, int i) {
    return i == 0 ? 1LL : (i == 1 ? d.sy : d.sz);
}

template <int STORE>
__device__ __forceinline__ void load_p(const YBuf<STORE> &Y, const Dims &d, long long idx, float p[3]) {
#pragma unroll
    for (int c = 0; c < 3; c++) p[c] = Store<STORE>::ld(Y.p + c * d.n + idx);
}

template <int STORE>
__device__ __forceinline__ void load_q(const YBuf<STORE> &Y, const Dims &d, long long idx, float q[6]) {
#pragma unroll
    for (int c = 0; c < 6; c++) q[c] = Store<STORE>::ld(Y.q + c * d.n + idx);
}

template <int STORE>
__device__ __forceinline__ void load_v(const XBuf<STORE> &X, const Dims &d, long long idx, float v[3]) {
#pragma unroll
    for (int c = 0; c < 3; c++) v[c] = Store<STORE>::ld(X.v + c * d.n + idx);
}

__device__ __forceinline__ void load_hist(const uint16_t *hist, long long idx, uint32_t hw[4]) {
    uint4 w = *reinterpret_cast<const uint4 *>(hist + 8 * idx);
    hw[0] = w.x;
    hw[1] = w.y;
    hw[2] = w.z;
    hw[3] = w.w;
}

// u+ at position s from the iterate (X, Y)
template <int STORE>
__device__ __forceinline__ float primal_u_at(const XBuf<STORE> &X, const YBuf<STORE> &Y, const uint16_t *hist,
                                             const Dims &d, const Coef &cf, const Pos &s) {
    float p[3], pm[3];
    load_p(Y, d, s.idx, p);
#pragma unroll
    for (int i = 0; i < 3; i++)
        pm[i] = s.mlo[i] ? Store<STORE>::ld(Y.p + i * d.n + s.idx - axis_stride(d, i)) : 0.0f;
    uint32_t hw[4];
    load_hist(hist, s.idx, hw);
    return primal_u(X.u[s.idx], p, pm, s.mlo, s.mhi, is_frozen(d, s.x, s.y, s.z), hw, cf);
}

// v+ at position s (rounded to the storage precision)
template <int STORE>
__device__ __forceinline__ void primal_v_at(const XBuf<STORE> &X, const YBuf<STORE> &Y, const Dims &d,
                                            const Coef &cf, const Pos &s, float vout[3]) {
    float v[3], p[3], q[6], qn[3][3];
    load_v(X, d, s.idx, v);
    load_p(Y, d, s.idx, p);
    load_q(Y, d, s.idx, q);
#pragma unroll
    for (int j = 0; j < 3; j++) {
        long long nb = s.idx + axis_stride(d, j);
#pragma unroll
        for (int i = 0; i < 3; i++)
            qn[i][j] = s.mhi[j] ? Store<STORE>::ld(Y.q + qslot(i, j) * d.n + nb) : 0.0f;
    }
    primal_v(vout, v, p, q, qn, s.mlo, s.mhi, cf);
#pragma unroll
    for (int i = 0; i < 3; i++) vout[i] = rnd<STORE>(vout[i]);
}

}  // namespace tgv
