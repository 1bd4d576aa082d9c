// Solver kernels, one thread per voxel, neighbours gathered through the
// caches: the dual step D, the primal step P and the fused step F
// (P then D in one pass, recomputing the primal values the dual needs at
// the six face neighbours).  These are the baseline kernels; they define
// the reference bits the tiled kernels must reproduce.
#include "fields.h"
#include "internal.h"

namespace tgv {

// D: Y <- dual(Y, 2 Xc - Xp), in place (each voxel reads only its own p, q)
template <int STORE>
__global__ void __launch_bounds__(256) k_dual(XBuf<STORE> Xc, XBuf<STORE> Xp, YBuf<STORE> Y, Dims d, Coef cf) {
    int x = blockIdx.x * blockDim.x + threadIdx.x;
    int y = blockIdx.y * blockDim.y + threadIdx.y;
    int z = blockIdx.z;
    if (x >= d.nx || y >= d.ny) return;
    Pos s = make_pos(d, x, y, z);
    float ub = 2.0f * Xc.u[s.idx] - Xp.u[s.idx];
    float ub_hi[3];
#pragma unroll
    for (int i = 0; i < 3; i++) {
        long long nb = s.idx + axis_stride(d, i);
        ub_hi[i] = s.mhi[i] ? (2.0f * Xc.u[nb] - Xp.u[nb]) : 0.0f;
    }
    float vc[3], vp[3], vb[3], vb_lo[3][3];
    load_v(Xc, d, s.idx, vc);
    load_v(Xp, d, s.idx, vp);
#pragma unroll
    for (int i = 0; i < 3; i++) vb[i] = 2.0f * vc[i] - vp[i];
#pragma unroll
    for (int j = 0; j < 3; j++) {
        long long nb = s.idx - axis_stride(d, j);
#pragma unroll
        for (int i = 0; i < 3; i++)
            vb_lo[j][i] = s.mlo[j] ? (2.0f * Store<STORE>::ld(Xc.v + i * d.n + nb) -
                                      Store<STORE>::ld(Xp.v + i * d.n + nb))
                                   : 0.0f;
    }
    float p[3], q[6];
    load_p(Y, d, s.idx, p);
    load_q(Y, d, s.idx, q);
    dual_pq(p, q, ub, ub_hi, vb, vb_lo, s.mlo, s.mhi, cf);
#pragma unroll
    for (int c = 0; c < 3; c++) Store<STORE>::st(Y.p + c * d.n + s.idx, p[c]);
#pragma unroll
    for (int c = 0; c < 6; c++) Store<STORE>::st(Y.q + c * d.n + s.idx, q[c]);
}

// P: Xn <- primal(Xc, Y)
template <int STORE>
__global__ void __launch_bounds__(256) k_primal(XBuf<STORE> Xc, YBuf<STORE> Y, XBuf<STORE> Xn,
                                                const uint16_t *__restrict__ hist, Dims d, Coef cf) {
    int x = blockIdx.x * blockDim.x + threadIdx.x;
    int y = blockIdx.y * blockDim.y + threadIdx.y;
    int z = blockIdx.z;
    if (x >= d.nx || y >= d.ny) return;
    Pos s = make_pos(d, x, y, z);
    Xn.u[s.idx] = primal_u_at(Xc, Y, hist, d, cf, s);
    float vo[3];
    primal_v_at(Xc, Y, d, cf, s, vo);
#pragma unroll
    for (int c = 0; c < 3; c++) Store<STORE>::st(Xn.v + c * d.n + s.idx, vo[c]);
}

// F: (Xn, Yn) <- (primal(Xc, Yc), dual(Yc, 2 Xn - Xc))
template <int STORE>
__global__ void __launch_bounds__(256) k_fused_ref(XBuf<STORE> Xc, YBuf<STORE> Yc, XBuf<STORE> Xn, YBuf<STORE> Yn,
                                                   const uint16_t *__restrict__ hist, Dims d, Coef cf) {
    int x = blockIdx.x * blockDim.x + threadIdx.x;
    int y = blockIdx.y * blockDim.y + threadIdx.y;
    int z = blockIdx.z;
    if (x >= d.nx || y >= d.ny) return;
    Pos s = make_pos(d, x, y, z);
    const int cc[3] = {x, y, z};
    // primal values at x
    float u_new = primal_u_at(Xc, Yc, hist, d, cf, s);
    float v_new[3];
    primal_v_at(Xc, Yc, d, cf, s, v_new);
    float ub = 2.0f * u_new - Xc.u[s.idx];
    float vc[3], vb[3];
    load_v(Xc, d, s.idx, vc);
#pragma unroll
    for (int i = 0; i < 3; i++) vb[i] = 2.0f * v_new[i] - vc[i];
    // u+ at the upper face neighbours
    float ub_hi[3];
#pragma unroll
    for (int i = 0; i < 3; i++) {
        if (s.mhi[i]) {
            int c2[3] = {cc[0], cc[1], cc[2]};
            c2[i] += 1;
            Pos t = make_pos(d, c2[0], c2[1], c2[2]);
            float un = primal_u_at(Xc, Yc, hist, d, cf, t);
            ub_hi[i] = 2.0f * un - Xc.u[t.idx];
        } else {
            ub_hi[i] = 0.0f;
        }
    }
    // v+ at the lower face neighbours
    float vb_lo[3][3];
#pragma unroll
    for (int j = 0; j < 3; j++) {
        if (s.mlo[j]) {
            int c2[3] = {cc[0], cc[1], cc[2]};
            c2[j] -= 1;
            Pos t = make_pos(d, c2[0], c2[1], c2[2]);
            float vn[3], vo[3];
            primal_v_at(Xc, Yc, d, cf, t, vn);
            load_v(Xc, d, t.idx, vo);
#pragma unroll
            for (int i = 0; i < 3; i++) vb_lo[j][i] = 2.0f * vn[i] - vo[i];
        } else {
#pragma unroll
            for (int i = 0; i < 3; i++) vb_lo[j][i] = 0.0f;
        }
    }
    float p[3], q[6];
    load_p(Yc, d, s.idx, p);
    load_q(Yc, d, s.idx, q);
    dual_pq(p, q, ub, ub_hi, vb, vb_lo, s.mlo, s.mhi, cf);
    Xn.u[s.idx] = u_new;
#pragma unroll
    for (int c = 0; c < 3; c++) Store<STORE>::st(Xn.v + c * d.n + s.idx, v_new[c]);
#pragma unroll
    for (int c = 0; c < 3; c++) Store<STORE>::st(Yn.p + c * d.n + s.idx, p[c]);
#pragma unroll
    for (int c = 0; c < 6; c++) Store<STORE>::st(Yn.q + c * d.n + s.idx, q[c]);
}

static dim3 ref_grid(const Dims &d) { return dim3((d.nx + 63) / 64, (d.ny + 3) / 4, d.nz); }

template <int STORE>
static void launch_ref_t(int kind, const SolveBufs &b, const Dims &d, const Coef &cf, hipStream_t s) {
    XBuf<STORE> Xc{b.xc_u, (typename Store<STORE>::T *)b.xc_v};
    XBuf<STORE> Xo{b.xo_u, (typename Store<STORE>::T *)b.xo_v};
    YBuf<STORE> Yc{(typename Store<STORE>::T *)b.yc_p, (typename Store<STORE>::T *)b.yc_q};
    YBuf<STORE> Yo{(typename Store<STORE>::T *)b.yo_p, (typename Store<STORE>::T *)b.yo_q};
    dim3 blk(64, 4, 1);
    if (kind == KIND_DUAL)
        hipLaunchKernelGGL(k_dual<STORE>, ref_grid(d), blk, 0, s, Xc, Xo, Yc, d, cf);
    else if (kind == KIND_PRIMAL)
        hipLaunchKernelGGL(k_primal<STORE>, ref_grid(d), blk, 0, s, Xc, Yc, Xo, b.hist, d, cf);
    else
        hipLaunchKernelGGL(k_fused_ref<STORE>, ref_grid(d), blk, 0, s, Xc, Yc, Xo, Yo, b.hist, d, cf);
}

void launch_ref(int kind, int storage, const SolveBufs &b, const Dims &d, const Coef &cf, hipStream_t s) {
    if (storage == 0) launch_ref_t<0>(kind, b, d, cf, s);
    else if (storage == 1) launch_ref_t<1>(kind, b, d, cf, s);
    else launch_ref_t<2>(kind, b, d, cf, s);
}

}  // namespace tgv
