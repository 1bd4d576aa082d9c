// Per-voxel arithmetic of the TGV-L1 primal-dual iteration (Eq. 2, Eq. 3,
// Sec. 3.2) shared by every solver kernel, so that the fused and the split
// schedules produce identical bits.  All code is compiled with
// -ffp-contract=off: each float operation rounds on its own.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

namespace tgv {

// ---------------------------------------------------------------------------
// storage precision of v, p, q (u is always float32)
// ---------------------------------------------------------------------------
struct bf16_t {
    uint16_t bits;
};

template <int STORE>
struct Store;

template <>
struct Store<0> {
    using T = float;
    static __device__ __forceinline__ float ld(const T *p) { return *p; }
    static __device__ __forceinline__ void st(T *p, float v) { *p = v; }
};

// float32 -> half, rounded once from the float32 value: the optimisation
// barrier keeps the compiler from folding a fused multiply-add that
// produced v into a mixed-precision instruction that rounds straight to
// half (one rounding instead of two), which some kernels would get and
// others not
__device__ __forceinline__ __half to_half(float v) {
    asm("" : "+v"(v));
    return __float2half_rn(v);
}

template <>
struct Store<1> {
    using T = __half;
    static __device__ __forceinline__ float ld(const T *p) { return __half2float(*p); }
    static __device__ __forceinline__ void st(T *p, float v) { *p = to_half(v); }
};

// float32 -> bfloat16 bits, rounded to nearest even by gfx950's conversion
// instruction (v_cvt_pk_bf16_f32); NaN stays NaN.  The same barrier as for
// half keeps every kernel rounding the float32 value once.
__device__ __forceinline__ uint16_t to_bf16_bits(float v) {
    asm("" : "+v"(v));
    return __builtin_bit_cast(uint16_t, (__bf16)v);
}

template <>
struct Store<2> {
    using T = bf16_t;
    static __device__ __forceinline__ float ld(const T *p) {
        return __uint_as_float(((uint32_t)p->bits) << 16);
    }
    static __device__ __forceinline__ void st(T *p, float v) { p->bits = to_bf16_bits(v); }
};

// ---------------------------------------------------------------------------
// block geometry
// ---------------------------------------------------------------------------
struct Dims {
    int nx, ny, nz, halo;
    long long n;        // nx * ny * nz
    long long sy, sz;   // strides of y and z (= nx, nx * ny)
};

__device__ __forceinline__ bool is_frozen(const Dims &d, int x, int y, int z) {
    int h = d.halo;
    return h > 0 && (x < h || y < h || z < h || x >= d.nx - h || y >= d.ny - h || z >= d.nz - h);
}

// a * b + c with one rounding.  The solver's products that feed a sum are
// fused explicitly (the library is built without automatic contraction,
// which the histogram rule needs); every solver kernel calls these same
// functions, so all schedules agree bit for bit.
__device__ __forceinline__ float madd(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// Solver constants (float32, as passed through the ABI)
struct Coef {
    float alpha0, alpha1, tau, sigma, taulam, taulam2;  // taulam = tau lambda, taulam2 = 2 tau lambda
    float c[8];  // bin centres, +inf in unused slots
    int tvl1;    // 1: the TV-L1 model of Eq. 1 (v stays 0, q unused)
};

// ---------------------------------------------------------------------------
// proximal map of lambda sum_k h_k |w - c_k| (step tau):
//   prox(ut) = max_{k=0..8} min(ut - tau lambda (2 S_k - W), c_k),
// (the g_k are formed by stepping down from g_0 by 2 tau lambda h_k),
// S_k = h_0 + ... + h_{k-1}, W = S_8, c_8 = +inf.  On the open interval
// between c_{k-1} and c_k the optimality condition gives w = ut - tau
// lambda (2 S_k - W); the max-min form selects that value or the centre
// where the subgradient contains 0.  Zero-count slots (and unused slots
// with c = +inf) are dominated and drop out.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float prox_hist(float ut, const uint32_t hw[4], const Coef &cf) {
    float h[8];
#pragma unroll
    for (int k = 0; k < 4; k++) {
        h[2 * k] = (float)(hw[k] & 0xffffu);
        h[2 * k + 1] = (float)(hw[k] >> 16);
    }
    float W = ((h[0] + h[1]) + (h[2] + h[3])) + ((h[4] + h[5]) + (h[6] + h[7]));  // exact: integers
    // g_k = ut - tau lambda (2 S_k - W), walked down from g_0 = ut + tau lambda W
    float g = madd(cf.taulam, W, ut);
    float best = fminf(g, cf.c[0]);
#pragma unroll
    for (int k = 1; k < 8; k++) {
        g = madd(-cf.taulam2, h[k - 1], g);
        best = fmaxf(best, fminf(g, cf.c[k]));
    }
    return fmaxf(best, madd(-cf.taulam, W, ut));
}

// projection onto {|y| <= alpha}: y / max(1, |y| / alpha), as y * alpha / |y|
// when |y| > alpha (one reciprocal square root); alpha = 0 gives 0
__device__ __forceinline__ void project3(float &a, float &b, float &c, float alpha) {
    float n2 = madd(c, c, madd(b, b, a * a));
    if (n2 > alpha * alpha) {
        float f = alpha * __builtin_amdgcn_rsqf(n2);
        a = a * f;
        b = b * f;
        c = c * f;
    }
}

// q is a symmetric 3x3 tensor (xx, yy, zz, xy, xz, yz); its norm counts the
// off-diagonal entries twice (Frobenius norm of the matrix)
__device__ __forceinline__ void project6(float q[6], float alpha) {
    float d = madd(q[2], q[2], madd(q[1], q[1], q[0] * q[0]));
    float o = madd(q[5], q[5], madd(q[4], q[4], q[3] * q[3]));
    float n2 = madd(2.0f, o, d);
    if (n2 > alpha * alpha) {
        float f = alpha * __builtin_amdgcn_rsqf(n2);
#pragma unroll
        for (int k = 0; k < 6; k++) q[k] = q[k] * f;
    }
}

// q slot of the (i, j) entry
__host__ __device__ constexpr int qslot(int i, int j) {
    return i == j ? i : ((i + j == 1) ? 3 : ((i + j == 2) ? 4 : 5));
}

// ---------------------------------------------------------------------------
// primal updates at one voxel y (Sec. 3.2):
//   u+ = prox(u + tau div p)  (u+ = u on frozen voxels),
//     div p(y) = sum_i ( [y_i < n_i - 1] p_i(y) - [y_i > 0] p_i(y - e_i) );
//   v+_i = v_i + tau ( [y_i < n_i - 1] p_i(y)
//                      + sum_j ( [y_j < n_j - 1] q_ij(y + e_j) - [y_j > 0] q_ij(y) ) ).
// The caller supplies the neighbour values (0 where the condition fails).
// ---------------------------------------------------------------------------
__device__ __forceinline__ float primal_u(float u, const float p[3], const float pm[3], const bool mlo[3],
                                          const bool mhi[3], bool frozen, const uint32_t hw[4], const Coef &cf) {
    float divp = 0.0f;
#pragma unroll
    for (int i = 0; i < 3; i++) {
        if (mhi[i]) divp = divp + p[i];
        if (mlo[i]) divp = divp - pm[i];
    }
    if (frozen) return u;
    return prox_hist(madd(cf.tau, divp, u), hw, cf);
}

// qn[i][j] = q_ij(y + e_j) (0 if y_j == n_j - 1); q = q(y)
__device__ __forceinline__ void primal_v(float vout[3], const float v[3], const float p[3], const float q[6],
                                         const float qn[3][3], const bool mlo[3], const bool mhi[3],
                                         const Coef &cf) {
    if (cf.tvl1) {
#pragma unroll
        for (int i = 0; i < 3; i++) vout[i] = v[i];
        return;
    }
#pragma unroll
    for (int i = 0; i < 3; i++) {
        float w = mhi[i] ? p[i] : 0.0f;
#pragma unroll
        for (int j = 0; j < 3; j++) {
            if (mhi[j]) w = w + qn[i][j];
            if (mlo[j]) w = w - q[qslot(i, j)];
        }
        vout[i] = madd(cf.tau, w, v[i]);
    }
}

// ---------------------------------------------------------------------------
// dual updates at one voxel x (Sec. 3.2), from the over-relaxed primal
// values ubar = 2 u+ - u, vbar = 2 v+ - v:
//   p <- P_alpha1(p + sigma M.(grad ubar - vbar)),
//   q <- P_alpha0(q + sigma E(vbar)),
// grad forward with the last cell dropped, E from backward differences
// (0 on the first cell).  ub_hi[i] = ubar(x + e_i), vb_lo[j][i] = vbar_i(x - e_j).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void dual_pq(float p[3], float q[6], float ub, const float ub_hi[3], const float vb[3],
                                        const float vb_lo[3][3], const bool mlo[3], const bool mhi[3],
                                        const Coef &cf) {
    float g[3];
#pragma unroll
    for (int i = 0; i < 3; i++) g[i] = mhi[i] ? ((ub_hi[i] - ub) - vb[i]) : 0.0f;
    float a = madd(cf.sigma, g[0], p[0]);
    float b = madd(cf.sigma, g[1], p[1]);
    float c = madd(cf.sigma, g[2], p[2]);
    project3(a, b, c, cf.alpha1);
    p[0] = a;
    p[1] = b;
    p[2] = c;
    if (cf.tvl1) return;  // no second-order term
    float dm[3][3];  // dm[i][j] = d-_j vbar_i
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) dm[i][j] = mlo[j] ? (vb[i] - vb_lo[j][i]) : 0.0f;
    float e[6];
    e[0] = dm[0][0];
    e[1] = dm[1][1];
    e[2] = dm[2][2];
    e[3] = 0.5f * (dm[0][1] + dm[1][0]);
    e[4] = 0.5f * (dm[0][2] + dm[2][0]);
    e[5] = 0.5f * (dm[1][2] + dm[2][1]);
#pragma unroll
    for (int k = 0; k < 6; k++) q[k] = madd(cf.sigma, e[k], q[k]);
    project6(q, cf.alpha0);
}

}  // namespace tgv
