// Fused TGV iteration on z-marching 2.5-D tiles.
//
// One workgroup owns a 64 x TY column tile of the block and walks a chunk of
// CZ planes along z.  Thread (tx, ty) owns the voxel column (x0 + tx,
// y0 + ty): the values of its column at the previous planes stay in
// registers, the in-plane neighbours it needs come through LDS.  The ring of
// columns around the tile (bottom and left rows: v is needed there; top and
// right rows: u is needed there; two corners: p and q only) is carried by
// three extra waves, so every thread owns exactly one column.  Per plane s the workgroup
//   1. publishes p_x, p_y of plane s and q of plane s-1 (LDS), barrier;
//   2. computes u+ at plane s and v+ at plane s-1 (same per-voxel
//      arithmetic as the reference kernels), publishes ubar of plane s-1 and
//      vbar of plane s-1, barrier;
//   3. computes the dual update of plane s-1 and stores u+, v+, p, q.
// Each input value is read from memory once per iteration (plus the ring);
// the next plane is in flight in registers while the current one is
// computed.  Barriers wait only for LDS traffic, so the prefetch stays in
// flight across them.  Results are bit-identical to the reference kernels.
#include "fields.h"
#include "internal.h"

#ifndef TILED_WAVES_PER_EU
#define TILED_WAVES_PER_EU 4
#endif


namespace tgv {

namespace {

constexpr int TX = 64;
// a lane offset past the end of every buffer: a raw buffer load there reads
// 0 and a store there is dropped, with no memory request (blocks of the
// tiled kernels stay below 2^31 bytes per buffer)
constexpr int LD_SKIP = (int)0x80000000u;
constexpr unsigned RSRC_WORD3 = 0x00020000u;  // raw buffer, 32-bit data format

// wait for this wave's LDS operations, then meet the workgroup; the memory
// clobber keeps the compiler from moving LDS accesses across it
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const void *p, long long bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes, (int)RSRC_WORD3);
}

// Field access through buffer descriptors: one descriptor per field array
// (uniform, in SGPRs); the lane supplies its column's byte offset and the
// uniform component/plane offset goes in the scalar offset.
template <int STORE>
struct Io;

template <>
struct Io<0> {
    template <int CP = 0>
    static __device__ __forceinline__ float ld(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
        return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, CP));
    }
    template <int CP = 0>
    static __device__ __forceinline__ void st(__amdgpu_buffer_rsrc_t r, int voff, int soff, float v) {
        __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, voff, soff, CP);
    }
};

template <>
struct Io<1> {
    template <int CP = 0>
    static __device__ __forceinline__ float ld(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
        unsigned short b = __builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, CP);
        return __half2float(__ushort_as_half(b));
    }
    template <int CP = 0>
    static __device__ __forceinline__ void st(__amdgpu_buffer_rsrc_t r, int voff, int soff, float v) {
        __builtin_amdgcn_raw_buffer_store_b16(__half_as_ushort(to_half(v)), r, voff, soff, CP);
    }
};

template <>
struct Io<2> {
    template <int CP = 0>
    static __device__ __forceinline__ float ld(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
        unsigned short b = __builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, CP);
        return __uint_as_float(((uint32_t)b) << 16);
    }
    template <int CP = 0>
    static __device__ __forceinline__ void st(__amdgpu_buffer_rsrc_t r, int voff, int soff, float v) {
        bf16_t t;
        Store<2>::st(&t, v);
        __builtin_amdgcn_raw_buffer_store_b16(t.bits, r, voff, soff, CP);
    }
};

struct Plane {
    float u, v[3], p[3], q[6];
    uint32_t h[4];
};

// q components the in-plane neighbours read: xx, yy, xy, xz, yz (q slots 0, 1, 3, 4, 5)
__device__ __forceinline__ int lq_of_slot(int slot) { return slot == 0 ? 0 : (slot == 1 ? 1 : slot - 1); }

template <int STORE, int TY, int SCP>
struct Tile {
    static constexpr int EX = TX + 2, EY = TY + 2, NE = EX * EY;
    static constexpr int SB = STORE == 0 ? 4 : 2;  // bytes per stored v/p/q element
    float *sPx, *sPy, *sQ, *sU, *sV;               // LDS planes (sQ: 5 x NE, sV: 3 x NE)
    __amdgpu_buffer_rsrc_t ru, rv, rp, rq, rh, wu, wv, wp, wq;
    int comp;                                      // component stride in bytes (n * SB)
    long long plane4, planeS, planeH;              // plane strides in bytes
    int v4, vS, vH;                                // the lane's column offsets in bytes
    const Dims *d;
    const Coef *cf;
    int e;                                         // LDS index of the lane's column
    bool core, needU, needV, in, active;
    bool mlo_x, mlo_y, mhi_x, mhi_y, fxy;
    int z0, zl;

    // Load plane s of the lane's column (every field, for every lane: the
    // loads stay branch-free so the compiler can issue them back to back).
    // With `on` false every offset is past the end of its buffer: the loads
    // are issued but read nothing (the raw buffer range check returns 0).
    __device__ __forceinline__ void load(Plane &L, int s, bool on = true) const {
        // planes past the block are clamped to the last one: their values are never used
        const int sc = s < d->nz ? s : d->nz - 1;
        const int o4 = (int)(plane4 * sc), oS = (int)(planeS * sc), oH = (int)(planeH * sc);
        const int v4 = on ? this->v4 : LD_SKIP, vS = on ? this->vS : LD_SKIP, vH = on ? this->vH : LD_SKIP;
        L.u = Io<0>::ld(ru, v4, o4);
        auto hv = __builtin_amdgcn_raw_buffer_load_b128(rh, vH, oH, 0);
        L.h[0] = hv[0];
        L.h[1] = hv[1];
        L.h[2] = hv[2];
        L.h[3] = hv[3];
#pragma unroll
        for (int c = 0; c < 3; c++) L.v[c] = Io<STORE>::ld(rv, vS, oS + c * comp);
#pragma unroll
        for (int c = 0; c < 3; c++) L.p[c] = Io<STORE>::ld(rp, vS, oS + c * comp);
#pragma unroll
        for (int c = 0; c < 6; c++) L.q[c] = Io<STORE>::ld(rq, vS, oS + c * comp);
    }

    // One plane step: prev = plane s-1, cur = plane s, nxt <- plane s+1.
    // Carried values: UP1/UB1 = u+ and ubar of plane s-1, VB2 = vbar of plane s-2.
    __device__ __forceinline__ void step(const Plane &prev, const Plane &cur, Plane &nxt, int s, int s1, float &UP1,
                                         float &UB1, float VB2[3]) const {
        const bool have_s = s < d->nz;
        const bool do_u = s >= z0 && have_s;
        const int sv = s - 1;
        const bool do_v = sv >= max(z0 - 1, 0) && sv <= zl;
        const bool do_dual = sv >= z0 && sv <= zl;

        // ---- 1. publish p_x, p_y of plane s and q of plane s-1
        if (active) {
            sPx[e] = cur.p[0];
            sPy[e] = cur.p[1];
            sQ[0 * NE + e] = prev.q[0];
            sQ[1 * NE + e] = prev.q[1];
            sQ[2 * NE + e] = prev.q[3];
            sQ[3 * NE + e] = prev.q[4];
            sQ[4 * NE + e] = prev.q[5];
        }
        // prefetch plane s+1, issued at every step (reading nothing past the
        // chunk) and after the plane in use is published: the memory counter
        // sees the same operations on every path, so a wait for the plane in
        // use never waits for the prefetch in flight
        load(nxt, s + 1, s + 1 <= s1);
        lds_barrier();

        // ---- 2. primal updates: u+ at plane s, v+ at plane s-1
        float UP = 0.0f, UB = 0.0f, VB[3] = {0.0f, 0.0f, 0.0f}, VP[3] = {0.0f, 0.0f, 0.0f};
        const bool zlo_s = s > 0, zhi_s = s < d->nz - 1;
        const bool zlo_v = sv > 0, zhi_v = sv < d->nz - 1;
        if (needU && do_u) {
            const bool fz = d->halo > 0 && (s < d->halo || s >= d->nz - d->halo);
            float pm[3];
            const float lx = sPx[e - 1], ly = sPy[e - EX];
            pm[0] = mlo_x ? lx : 0.0f;
            pm[1] = mlo_y ? ly : 0.0f;
            pm[2] = zlo_s ? prev.p[2] : 0.0f;
            const bool mlo[3] = {mlo_x, mlo_y, zlo_s}, mhi[3] = {mhi_x, mhi_y, zhi_s};
            UP = primal_u(cur.u, cur.p, pm, mlo, mhi, fxy || fz, cur.h, *cf);
            UB = 2.0f * UP - cur.u;
        }
        if (needV && do_v) {
            float qn[3][3];
#pragma unroll
            for (int i = 0; i < 3; i++) {
                const float ax = sQ[lq_of_slot(qslot(i, 0)) * NE + e + 1];
                const float ay = sQ[lq_of_slot(qslot(i, 1)) * NE + e + EX];
                qn[i][0] = mhi_x ? ax : 0.0f;
                qn[i][1] = mhi_y ? ay : 0.0f;
                qn[i][2] = zhi_v ? cur.q[qslot(i, 2)] : 0.0f;
            }
            const bool mlo[3] = {mlo_x, mlo_y, zlo_v}, mhi[3] = {mhi_x, mhi_y, zhi_v};
            primal_v(VP, prev.v, prev.p, prev.q, qn, mlo, mhi, *cf);
#pragma unroll
            for (int i = 0; i < 3; i++) {
                VP[i] = rnd<STORE>(VP[i]);
                VB[i] = 2.0f * VP[i] - prev.v[i];
            }
        }
        if (needU) sU[e] = UB1;
        if (needV) {
            sV[0 * NE + e] = VB[0];
            sV[1 * NE + e] = VB[1];
            sV[2 * NE + e] = VB[2];
        }
        lds_barrier();

        // ---- 3. dual update of plane s-1 and stores
        float p[3] = {0.0f, 0.0f, 0.0f};
        float q[6] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
        const bool made = core && do_dual;
        if (made) {
            const bool mlo[3] = {mlo_x, mlo_y, zlo_v}, mhi[3] = {mhi_x, mhi_y, zhi_v};
            float ub_hi[3], vb_lo[3][3];
            const float ux = sU[e + 1], uy = sU[e + EX];
            ub_hi[0] = mhi_x ? ux : 0.0f;
            ub_hi[1] = mhi_y ? uy : 0.0f;
            ub_hi[2] = zhi_v ? UB : 0.0f;
#pragma unroll
            for (int i = 0; i < 3; i++) {
                const float bx = sV[i * NE + e - 1], by = sV[i * NE + e - EX];
                vb_lo[0][i] = mlo_x ? bx : 0.0f;
                vb_lo[1][i] = mlo_y ? by : 0.0f;
                vb_lo[2][i] = zlo_v ? VB2[i] : 0.0f;
            }
#pragma unroll
            for (int c = 0; c < 3; c++) p[c] = prev.p[c];
#pragma unroll
            for (int c = 0; c < 6; c++) q[c] = prev.q[c];
            dual_pq(p, q, UB1, ub_hi, VB, vb_lo, mlo, mhi, *cf);
        }
        {
            // the stores are issued at every step; lanes without a result get
            // an offset past the end of the buffer, which drops the store
            const int svc = sv > 0 ? sv : 0;
            const int o4 = (int)(plane4 * svc), oS = (int)(planeS * svc);
            const int a4 = (made && in) ? v4 : LD_SKIP, aS = (made && in) ? vS : LD_SKIP;
            Io<0>::st<SCP>(wu, a4, o4, UP1);
#pragma unroll
            for (int c = 0; c < 3; c++) Io<STORE>::template st<SCP>(wv, aS, oS + c * comp, VP[c]);
#pragma unroll
            for (int c = 0; c < 3; c++) Io<STORE>::template st<SCP>(wp, aS, oS + c * comp, p[c]);
#pragma unroll
            for (int c = 0; c < 6; c++) Io<STORE>::template st<SCP>(wq, aS, oS + c * comp, q[c]);
        }
        UP1 = UP;
        UB1 = UB;
        VB2[0] = VB[0];
        VB2[1] = VB[1];
        VB2[2] = VB[2];
    }
};

}  // namespace

// LDS planes of one tile
template <int TY>
struct TileLds {
    static constexpr int NE = (TX + 2) * (TY + 2);
    float sPx[NE], sPy[NE];
    float sQ[5 * NE];
    float sU[NE];
    float sV[3 * NE];
};

// One fused iteration on tile (tix, tiy, tiz) of a block: X/Y current
// buffers in, Xn/Yn out.  Every thread of the workgroup must call this
// (it contains workgroup barriers).
template <int STORE, int TY, int SCP>
__device__ __forceinline__ void run_tile(TileLds<TY> &lds, const XBuf<STORE> &Xc, const YBuf<STORE> &Yc,
                                         const XBuf<STORE> &Xn, const YBuf<STORE> &Yn, const uint16_t *hist,
                                         const Dims &d, const Coef &cf, int CZ, int tix, int tiy, int tiz) {
    using T = Tile<STORE, TY, SCP>;
    constexpr int EX = T::EX;
    const int x0 = tix * TX, y0 = tiy * TY, z0 = tiz * CZ;

    // Each thread owns one column of the extended tile.  Waves 0..TY-1: the
    // tile's rows (dual update and stores); wave TY: the row below (v+
    // needed); wave TY+1: the row above (u+ needed); wave TY+2: the left
    // column (v+), the right column (u+) and the two corners read by the
    // ring (p and q only).
    const int w = threadIdx.x / TX, lane = threadIdx.x & (TX - 1);
    int px = -2, py = -2;
    bool core = false, needU = false, needV = false, active = true;
    if (w < TY) {
        px = x0 + lane; py = y0 + w; core = needU = needV = true;
    } else if (w == TY) {
        px = x0 + lane; py = y0 - 1; needV = true;
    } else if (w == TY + 1) {
        px = x0 + lane; py = y0 + TY; needU = true;
    } else {
        if (lane < TY) { px = x0 - 1; py = y0 + lane; needV = true; }
        else if (lane < 2 * TY) { px = x0 + TX; py = y0 + lane - TY; needU = true; }
        else if (lane == 2 * TY) { px = x0 - 1; py = y0 + TY; }
        else if (lane == 2 * TY + 1) { px = x0 + TX; py = y0 - 1; }
        else active = false;
    }
    const bool in = active && px >= 0 && py >= 0 && px < d.nx && py < d.ny;

    T t;
    t.sPx = lds.sPx;
    t.sPy = lds.sPy;
    t.sQ = lds.sQ;
    t.sU = lds.sU;
    t.sV = lds.sV;
    t.d = &d;
    t.cf = &cf;
    t.in = in;
    t.active = active;
    // columns outside the block compute nothing (their loads are clamped to
    // column 0 and their results are never read)
    t.needU = needU && in;
    t.needV = needV && in;
    t.core = core && in;
    t.e = active ? (py - y0 + 1) * EX + (px - x0 + 1) : 0;
    t.mlo_x = px > 0;
    t.mlo_y = py > 0;
    t.mhi_x = px < d.nx - 1;
    t.mhi_y = py < d.ny - 1;
    t.fxy = d.halo > 0 && (px < d.halo || py < d.halo || px >= d.nx - d.halo || py >= d.ny - d.halo);
    t.z0 = z0;
    t.zl = min(z0 + CZ, d.nz) - 1;
    const long long col = in ? (long long)px + d.sy * py : 0;
    t.v4 = (int)(col * 4);
    t.vS = (int)(col * T::SB);
    t.vH = (int)(col * 16);
    t.comp = (int)(d.n * T::SB);
    t.plane4 = d.sz * 4;
    t.planeS = d.sz * T::SB;
    t.planeH = d.sz * 16;
    t.ru = rsrc(Xc.u, d.n * 4);
    t.rv = rsrc(Xc.v, 3 * d.n * T::SB);
    t.rp = rsrc(Yc.p, 3 * d.n * T::SB);
    t.rq = rsrc(Yc.q, 6 * d.n * T::SB);
    t.rh = rsrc(hist, d.n * 16);
    t.wu = rsrc(Xn.u, d.n * 4);
    t.wv = rsrc(Xn.v, 3 * d.n * T::SB);
    t.wp = rsrc(Yn.p, 3 * d.n * T::SB);
    t.wq = rsrc(Yn.q, 6 * d.n * T::SB);

    const int s0 = max(z0 - 1, 0);
    const int s1 = t.zl + 1;  // may equal nz: that step loads nothing
    // three-plane rotation, one plane in flight: (prev, cur, next) = (A, B, C), (B, C, A), (C, A, B)
    Plane A, B, C;
    float UP1 = 0.0f, UB1 = 0.0f, VB2[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int c = 0; c < 3; c++) A.p[c] = A.v[c] = 0.0f;
#pragma unroll
    for (int c = 0; c < 6; c++) A.q[c] = 0.0f;
    t.load(B, s0);
    // no early exit inside the unrolled loop: one or two trailing steps
    // past s1 load and store nothing, and the loop keeps one shape
    for (int s = s0; s <= s1; s += 3) {
        t.step(A, B, C, s, s1, UP1, UB1, VB2);
        t.step(B, C, A, s + 1, s1, UP1, UB1, VB2);
        t.step(C, A, B, s + 2, s1, UP1, UB1, VB2);
    }
}

// Occupancy target of the one-block kernel per configuration (measured):
// float32 storage with 64 x 8 tiles fits 80 VGPRs without spilling, which
// gives 6 waves per SIMD and two workgroups of 11 waves per CU; the other
// configurations are fastest with the default register budget.
constexpr int tiled_waves(int store, int ty) { return (store == 0 && ty == 8) ? 6 : TILED_WAVES_PER_EU; }

template <int STORE, int TY, int SCP>
__global__ void __launch_bounds__(TX *(TY + 3), tiled_waves(STORE, TY)) k_fused_tiled(XBuf<STORE> Xc, YBuf<STORE> Yc,
                                                                                  XBuf<STORE> Xn, YBuf<STORE> Yn,
                                                                                  const uint16_t *__restrict__ hist,
                                                                                  Dims d, Coef cf, int CZ, int ntx,
                                                                                  int nty, int ntz) {
    __shared__ TileLds<TY> lds;
    // XCD-aware tile order: workgroups are dealt round-robin to the 8 XCDs;
    // give each XCD a contiguous run of tiles so neighbours share its L2
    const int nb = ntx * nty * ntz;
    const int per = (nb + 7) / 8;
    const int L = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
    if (L >= nb) return;
    run_tile<STORE, TY, SCP>(lds, Xc, Yc, Xn, Yn, hist, d, cf, CZ, L % ntx, (L / ntx) % nty, L / (ntx * nty));
}

// ---------------------------------------------------------------------------
// batched fused iteration: many blocks in one persistent launch
// ---------------------------------------------------------------------------
// Workgroups pull tiles from a device work queue split into 8 segments (one
// per XCD, so the tiles of a block stay near each other's L2); a workgroup
// drains its own segment, then takes from the others.  Every tile of every
// block advances one iteration per launch; no workgroup waits on another.
template <int STORE, int TY>
__global__ void __launch_bounds__(TX *(TY + 3), TILED_WAVES_PER_EU) k_fused_batch(const BatchBlock *__restrict__ blocks,
                                                                                  const int4 *__restrict__ tiles,
                                                                                  int ntiles, int *counters, Coef cf,
                                                                                  int flip) {
    __shared__ TileLds<TY> lds;
    __shared__ int s_tile;
    const int seg_len = (ntiles + 7) / 8;
    const int home = (int)(blockIdx.x % 8);
    for (int k = 0; k < 8; k++) {
        const int seg = (home + k) & 7;
        const int seg_end = min(seg_len * (seg + 1), ntiles);
        while (true) {
            if (threadIdx.x == 0) s_tile = seg * seg_len + atomicAdd(&counters[seg], 1);
            lds_barrier();
            const int ti = s_tile;
            lds_barrier();  // everyone has read s_tile before it is rewritten
            if (ti >= seg_end) break;
            const int4 tr = tiles[ti];
            const BatchBlock &bb = blocks[tr.x];
            const int xc = bb.xc ^ flip, yc = bb.yc ^ flip;
            XBuf<STORE> Xc{bb.u[xc], (typename Store<STORE>::T *)bb.v[xc]};
            XBuf<STORE> Xn{bb.u[xc ^ 1], (typename Store<STORE>::T *)bb.v[xc ^ 1]};
            YBuf<STORE> Yc{(typename Store<STORE>::T *)bb.p[yc], (typename Store<STORE>::T *)bb.q[yc]};
            YBuf<STORE> Yn{(typename Store<STORE>::T *)bb.p[yc ^ 1], (typename Store<STORE>::T *)bb.q[yc ^ 1]};
            run_tile<STORE, TY, 0>(lds, Xc, Yc, Xn, Yn, bb.hist, bb.d, cf, bb.cz, tr.y & 0xffff, tr.y >> 16, tr.z);
            lds_barrier();  // the tile's LDS reads are done before the next tile writes
        }
    }
}

__global__ void k_reset_counters(int *counters) {
    if (threadIdx.x < 8) counters[threadIdx.x] = 0;
}

void launch_reset_counters(int *counters, hipStream_t s) {
    hipLaunchKernelGGL(k_reset_counters, dim3(1), dim3(64), 0, s, counters);
}

template <int STORE, int TY, int SCP>
static void launch_tiled_ty(const SolveBufs &b, const Dims &d, const Coef &cf, int cz, hipStream_t s) {
    XBuf<STORE> Xc{b.xc_u, (typename Store<STORE>::T *)b.xc_v};
    XBuf<STORE> Xo{b.xo_u, (typename Store<STORE>::T *)b.xo_v};
    YBuf<STORE> Yc{(typename Store<STORE>::T *)b.yc_p, (typename Store<STORE>::T *)b.yc_q};
    YBuf<STORE> Yo{(typename Store<STORE>::T *)b.yo_p, (typename Store<STORE>::T *)b.yo_q};
    int ntx = (d.nx + TX - 1) / TX, nty = (d.ny + TY - 1) / TY, ntz = (d.nz + cz - 1) / cz;
    int nb = ntx * nty * ntz;
    int per = (nb + 7) / 8;
    hipLaunchKernelGGL((k_fused_tiled<STORE, TY, SCP>), dim3(8 * per), dim3(TX * (TY + 3)), 0, s, Xc, Yc, Xo, Yo, b.hist, d,
                       cf, cz, ntx, nty, ntz);
}

template <int STORE, int SCP>
static void launch_tiled_t(const SolveBufs &b, const Dims &d, const Coef &cf, int ty, int cz, hipStream_t s) {
    if (ty == 4) launch_tiled_ty<STORE, 4, SCP>(b, d, cf, cz, s);
    else if (ty == 12) launch_tiled_ty<STORE, 12, SCP>(b, d, cf, cz, s);
    else launch_tiled_ty<STORE, 8, SCP>(b, d, cf, cz, s);
}

bool tiled_shape_ok(int ty, int cz) { return (ty == 4 || ty == 8 || ty == 12) && cz >= 1; }

template <int STORE>
static void launch_batch_t(const BatchBlock *blocks, const int4 *tiles, int ntiles, int *counters, const Coef &cf,
                           int ty, int flip, int grid, hipStream_t s) {
    if (ty == 4)
        hipLaunchKernelGGL((k_fused_batch<STORE, 4>), dim3(grid), dim3(TX * 7), 0, s, blocks, tiles, ntiles, counters,
                           cf, flip);
    else if (ty == 7)  // single passes of a two-iteration batch, on its 64 x 7 tile table
        hipLaunchKernelGGL((k_fused_batch<STORE, 7>), dim3(grid), dim3(TX * 10), 0, s, blocks, tiles, ntiles,
                           counters, cf, flip);
    else if (ty == 6)  // the same on a 64 x 6 table
        hipLaunchKernelGGL((k_fused_batch<STORE, 6>), dim3(grid), dim3(TX * 9), 0, s, blocks, tiles, ntiles,
                           counters, cf, flip);
    else if (ty == 12)
        hipLaunchKernelGGL((k_fused_batch<STORE, 12>), dim3(grid), dim3(TX * 15), 0, s, blocks, tiles, ntiles,
                           counters, cf, flip);
    else
        hipLaunchKernelGGL((k_fused_batch<STORE, 8>), dim3(grid), dim3(TX * 11), 0, s, blocks, tiles, ntiles,
                           counters, cf, flip);
}

// resident workgroups per CU of the batched kernel (registers and LDS)
template <int STORE, int TY>
static int batch_per_cu_t() {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_fused_batch<STORE, TY>, TX * (TY + 3), 0) != hipSuccess)
        return 1;
    return nb > 0 ? nb : 1;
}

template <int STORE>
static int batch_per_cu_s(int ty) {
    return ty == 4    ? batch_per_cu_t<STORE, 4>()
           : ty == 12 ? batch_per_cu_t<STORE, 12>()
           : ty == 7  ? batch_per_cu_t<STORE, 7>()
           : ty == 6  ? batch_per_cu_t<STORE, 6>()
                      : batch_per_cu_t<STORE, 8>();
}

int batch_blocks_per_cu(int storage, int ty) {
    return storage == 0 ? batch_per_cu_s<0>(ty) : (storage == 1 ? batch_per_cu_s<1>(ty) : batch_per_cu_s<2>(ty));
}

void launch_batch(int storage, const BatchBlock *blocks, const int4 *tiles, int ntiles, int *counters, const Coef &cf,
                  int ty, int flip, int grid, hipStream_t s) {
    hipLaunchKernelGGL(k_reset_counters, dim3(1), dim3(64), 0, s, counters);
    if (storage == 0) launch_batch_t<0>(blocks, tiles, ntiles, counters, cf, ty, flip, grid, s);
    else if (storage == 1) launch_batch_t<1>(blocks, tiles, ntiles, counters, cf, ty, flip, grid, s);
    else launch_batch_t<2>(blocks, tiles, ntiles, counters, cf, ty, flip, grid, s);
}

// resident workgroups per CU of the one-block kernel
template <int STORE, int TY, int SCP>
static int tiled_per_cu_t() {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_fused_tiled<STORE, TY, SCP>, TX * (TY + 3), 0) != hipSuccess)
        return 1;
    return nb > 0 ? nb : 1;
}

template <int STORE, int SCP>
static int tiled_per_cu_s(int ty) {
    return ty == 4 ? tiled_per_cu_t<STORE, 4, SCP>()
                   : (ty == 12 ? tiled_per_cu_t<STORE, 12, SCP>() : tiled_per_cu_t<STORE, 8, SCP>());
}

int tiled_blocks_per_cu(int storage, int ty, const Dims &d) {
    if (stream_stores(storage, d))
        return storage == 0 ? tiled_per_cu_s<0, STORE_CP_STREAM>(ty)
                            : (storage == 1 ? tiled_per_cu_s<1, STORE_CP_STREAM>(ty) : tiled_per_cu_s<2, STORE_CP_STREAM>(ty));
    return storage == 0 ? tiled_per_cu_s<0, 0>(ty) : (storage == 1 ? tiled_per_cu_s<1, 0>(ty) : tiled_per_cu_s<2, 0>(ty));
}

// Planes per z-chunk of the one-block kernel: the depth up to 32 that
// minimises rounds of resident workgroups x (cz + 2) plane steps.  A block
// with enough tiles keeps 32 planes (256^3: 1024 tiles, two full rounds;
// deeper chunks were slower there, as neighbouring tiles drift further
// apart); a small block gets short chunks, so that its tiles fill the GPU
// instead of a few workgroups walking 32 planes each (64^3: 2 planes, 51 us
// per iteration with 32).
int choose_tile_z(const Dims &d, int ty, int slots) {
    const long long per_chunk = (long long)((d.nx + TX - 1) / TX) * ((d.ny + ty - 1) / ty);
    const int hi = d.nz < 32 ? d.nz : 32;
    long long best = -1;
    int best_cz = hi;
    for (int cz = hi; cz >= 1; cz--) {
        const long long tiles = per_chunk * ((d.nz + cz - 1) / cz);
        const long long rounds = (tiles + slots - 1) / slots;
        const long long cost = rounds * (cz + 2);
        if (best < 0 || cost < best) {
            best = cost;
            best_cz = cz;
        }
    }
    return best_cz;
}

bool tiled_fits(const Dims &d) {
    // every byte offset (component * n + plane * nx * ny, in 4-byte elements) must fit a signed 32-bit offset
    return d.n * 24 < (1LL << 31);
}

void launch_tiled(int storage, const SolveBufs &b, const Dims &d, const Coef &cf, int ty, int cz, hipStream_t s) {
    if (!tiled_fits(d)) {
        launch_ref(KIND_FUSED, storage, b, d, cf, s);
        return;
    }
    if (stream_stores(storage, d)) {
        if (storage == 0) launch_tiled_t<0, STORE_CP_STREAM>(b, d, cf, ty, cz, s);
        else if (storage == 1) launch_tiled_t<1, STORE_CP_STREAM>(b, d, cf, ty, cz, s);
        else launch_tiled_t<2, STORE_CP_STREAM>(b, d, cf, ty, cz, s);
    } else {
        if (storage == 0) launch_tiled_t<0, 0>(b, d, cf, ty, cz, s);
        else if (storage == 1) launch_tiled_t<1, 0>(b, d, cf, ty, cz, s);
        else launch_tiled_t<2, 0>(b, d, cf, ty, cz, s);
    }
}

}  // namespace tgv
