// Two fused iterations per pass over HBM (temporal blocking along z).
//
// A workgroup owns a 64 x TY column tile and walks a chunk of planes along
// z, like the one-iteration kernel, but runs two iterations in one sweep:
//   stage A computes iteration n from the state in memory on the tile and a
//     one-column ring around it (full update), with the partial primal
//     updates its dual step needs on a second ring;
//   stage B computes iteration n+1 on the tile, two planes behind stage A,
//     from stage A's results held in registers, and writes them to memory.
// Each input is read from HBM once and each output written once per two
// iterations.  Stage B needs stage A's results on the tile plus the first
// ring, stage A needs the state on the tile plus two rings; the rings are
// carried by five extra waves (two row waves per ring and one for the
// columns and corners).  Stage B takes each plane's histograms from LDS,
// where stage A left them two steps earlier.  Both stages use the per-voxel arithmetic of the
// one-iteration kernels, so two iterations here are bit-identical to two
// iterations there.
#include "fields.h"
#include "internal.h"

#ifndef TILED2_WAVES_PER_EU
#define TILED2_WAVES_PER_EU 3
#endif


namespace tgv {

namespace {

constexpr int TX = 64;
constexpr unsigned RSRC_WORD3 = 0x00020000u;

__device__ __forceinline__ void lds_barrier2() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc2(const void *p, long long bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes, (int)RSRC_WORD3);
}

// All fields of a state in one allocation of at most 2 GiB: one buffer
// descriptor serves every field, each field's byte offset from `base` goes
// into the scalar offset (frees the scalar registers of seven descriptors).
// The 2 GiB bound keeps a skipped load (lane offset 2^31) past the end.
struct Span {
    const void *base;
    int bytes;
    int u0, v0, p0, q0;  // current iterate
    int u1, v1, p1, q1;  // next iterate
};

template <int STORE>
struct Io2;
template <>
struct Io2<0> {
    static __device__ __forceinline__ float ld(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
        return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
    }
    template <int CP>
    static __device__ __forceinline__ void st(__amdgpu_buffer_rsrc_t r, int voff, int soff, float v) {
        __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, voff, soff, CP);
    }
};
template <>
struct Io2<1> {
    static __device__ __forceinline__ uint32_t raw(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
        return __builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, 0);
    }
    static __device__ __forceinline__ float cvt(uint32_t b) { return __half2float(__ushort_as_half((unsigned short)b)); }
    static __device__ __forceinline__ float ld(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
        return __half2float(__ushort_as_half(__builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, 0)));
    }
    template <int CP>
    static __device__ __forceinline__ void st(__amdgpu_buffer_rsrc_t r, int voff, int soff, float v) {
        __builtin_amdgcn_raw_buffer_store_b16(__half_as_ushort(to_half(v)), r, voff, soff, CP);
    }
};
template <>
struct Io2<2> {
    static __device__ __forceinline__ uint32_t raw(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
        return __builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, 0);
    }
    static __device__ __forceinline__ float cvt(uint32_t b) { return __uint_as_float(b << 16); }
    static __device__ __forceinline__ float ld(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
        return __uint_as_float(((uint32_t)__builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, 0)) << 16);
    }
    template <int CP>
    static __device__ __forceinline__ void st(__amdgpu_buffer_rsrc_t r, int voff, int soff, float v) {
        bf16_t t;
        Store<2>::st(&t, v);
        __builtin_amdgcn_raw_buffer_store_b16(t.bits, r, voff, soff, CP);
    }
};

// Fields a lane loads (bit mask).  A skipped field gets a lane offset past
// the end of its buffer, so the load returns 0 without a memory request
// (raw buffer range check).
enum : int {
    LD2_U = 1 << 0,
    LD2_V = 1 << 1,
    LD2_PX = 1 << 2,
    LD2_PY = 1 << 3,
    LD2_PZ = 1 << 4,
    LD2_Q0 = 1 << 5,  // q slot k: LD2_Q0 << k
    LD2_H = 1 << 11,
    LD2_P = LD2_PX | LD2_PY | LD2_PZ,
    LD2_Q = 63 * LD2_Q0,
    LD2_ALL = LD2_U | LD2_V | LD2_P | LD2_Q | LD2_H,
};
constexpr int LD2_SKIP = (int)0x80000000u;  // >= every buffer's size (below 2^31 for tiled blocks)

// the state of one column at one plane
struct Pl {
    float u, v[3], p[3], q[6];
};

__device__ __forceinline__ int lq2(int slot) { return slot == 0 ? 0 : (slot == 1 ? 1 : slot - 1); }

// LDS exchange planes of one stage over the (TX+4) x (TY+4) index space
template <int TY>
struct XLds {
    static constexpr int EX = TX + 4, NE = EX * (TY + 4);
    float sPx[NE], sPy[NE];
    float sQ[5 * NE];
    float sU[NE];
    float sV[3 * NE];
};

// histograms of the last three planes of stage A, for stage B (each lane
// reads back what it wrote two steps earlier)
template <int TY>
struct HLds {
    uint4 h[3][64 * (TY + 5)];
};

// One stage of one column: the z-pipeline of the one-iteration kernel,
// with its inputs handed in per plane and its dual results handed out.
struct Stage {
    bool needU, needV, full, active;  // roles of this column in this stage
    int z0, zl;                       // output planes of this stage
    float UP1, UB1, VB2[3];           // u+ and ubar of plane s-1, vbar of plane s-2
    float VP[3], VB[3], UP, UB;       // this plane step's primal results
};

}  // namespace

// Two fused iterations on tile (tix, tiy, tiz) of a block: Xc, Yc in, Xn, Yn
// out.  Every thread of the workgroup must call it (it holds barriers).
// TV: the TV-L1 model in float32 storage, whose v and q are zero in memory
// (the solve sets them so) and stay zero: they are neither loaded (a
// skipped load reads 0) nor stored.  Other TV-L1 solves run the TV = false
// kernels, which read and write those zeros.
template <int STORE, int TY, int SCP, bool TV = false, bool UNI = false>
__device__ __forceinline__ void run_tile2(XLds<TY> &la, XLds<TY> &lb, HLds<TY> &lh, const XBuf<STORE> &Xc,
                                          const YBuf<STORE> &Yc, const XBuf<STORE> &Xn, const YBuf<STORE> &Yn,
                                          const uint16_t *__restrict__ hist, const Dims &d, const Coef &cf, int CZ,
                                          int tix, int tiy, int tiz, const Span &sp = Span{}) {
    using L = XLds<TY>;
    constexpr int EX = L::EX, NE = L::NE;
    constexpr int SB = STORE == 0 ? 4 : 2;
    const int x0 = tix * TX, y0 = tiy * TY, z0 = tiz * CZ;
    const int zl = min(z0 + CZ, d.nz) - 1;

    // ---- the column this thread owns and its roles in both stages
    // waves 0..TY-1 core rows; TY: ring-1 row below; TY+1: ring-1 row above;
    // TY+2: ring-2 row below; TY+3: ring-2 row above; TY+4: the ring
    // columns, the rows' end columns and the two outer corners
    const int w = threadIdx.x / TX, lane = threadIdx.x & (TX - 1);
    // the tile's rows run both stages and set the length of every phase
    // between barriers: their waves issue first (256^3: 1 % faster)
    if (w < TY) __builtin_amdgcn_s_setprio(2);
    int px = -3, py = -3;
    // kind: 0 core, 1 ring-1, 2 ring-2 needing u+, 3 ring-2 needing v+, 4 ring-2 corner, -1 none
    int kind = -1;
    // Load masks (stage B loads nothing): the tile and the first ring read
    // every field; the second ring reads what stage A's partial updates
    // there use: v, p and q where v+ is formed (bottom row, left column);
    // u, p, the histogram and the q components the first ring's v+ takes
    // from it where u+ is formed (q_iy on the top row, q_ix on the right
    // column); p_x and q_iy (upper-left corner) or p_y and q_ix (lower-right).
    constexpr int Q_IX = LD2_Q0 << 0 | LD2_Q0 << 3 | LD2_Q0 << 4;  // xx, xy, xz
    constexpr int Q_IY = LD2_Q0 << 1 | LD2_Q0 << 3 | LD2_Q0 << 5;  // yy, xy, yz
    constexpr int M_V = LD2_V | LD2_P | LD2_Q, M_TOP = LD2_U | LD2_P | LD2_H | Q_IY,
                  M_RIGHT = LD2_U | LD2_P | LD2_H | Q_IX;
    int lm = 0;
    if (w < TY) { px = x0 + lane; py = y0 + w; kind = 0; lm = LD2_ALL; }
    else if (w == TY) { px = x0 + lane; py = y0 - 1; kind = 1; lm = LD2_ALL; }
    else if (w == TY + 1) { px = x0 + lane; py = y0 + TY; kind = 1; lm = LD2_ALL; }
    else if (w == TY + 2) { px = x0 + lane; py = y0 - 2; kind = 3; lm = M_V; }
    else if (w == TY + 3) { px = x0 + lane; py = y0 + TY + 1; kind = 2; lm = M_TOP; }
    else {
        int l = lane;
        if (l < TY) { px = x0 - 1; py = y0 + l; kind = 1; lm = LD2_ALL; }
        else if ((l -= TY) < TY) { px = x0 + TX; py = y0 + l; kind = 1; lm = LD2_ALL; }
        else if ((l -= TY) < 4) {
            px = (l & 1) ? x0 + TX : x0 - 1; py = (l & 2) ? y0 + TY : y0 - 1; kind = 1; lm = LD2_ALL;
        }
        else if ((l -= 4) < TY + 2) { px = x0 - 2; py = y0 - 1 + l; kind = 3; lm = M_V; }
        else if ((l -= TY + 2) < TY + 2) { px = x0 + TX + 1; py = y0 - 1 + l; kind = 2; lm = M_RIGHT; }
        else if ((l -= TY + 2) < 2) { px = l ? x0 + TX : x0 - 1; py = y0 - 2; kind = 3; lm = M_V; }
        else if ((l -= 2) < 2) { px = l ? x0 + TX : x0 - 1; py = y0 + TY + 1; kind = 2; lm = M_TOP; }
        else if ((l -= 2) < 2) {
            px = l ? x0 + TX + 1 : x0 - 2; py = l ? y0 - 2 : y0 + TY + 1; kind = 4;
            lm = l ? (LD2_PY | Q_IX) : (LD2_PX | Q_IY);
        }
    }
    const bool active = kind >= 0;
    const bool in = active && px >= 0 && py >= 0 && px < d.nx && py < d.ny;
    // 16-bit fields: every lane loads every field (lanes outside the block
    // read column 0, as in the one-iteration kernel); masked-off 16-bit loads
    // made both kernels slower
    const int lmask = STORE == 0 ? ((in ? lm : 0) & (TV ? ~(LD2_V | LD2_Q) : ~0)) : LD2_ALL;
    const int e = active ? (py - y0 + 2) * EX + (px - x0 + 2) : 0;
    const bool mlo_x = px > 0, mlo_y = py > 0, mhi_x = px < d.nx - 1, mhi_y = py < d.ny - 1;
    const bool fxy = d.halo > 0 && (px < d.halo || py < d.halo || px >= d.nx - d.halo || py >= d.ny - d.halo);

    // stage A: full on core + ring 1, partial on ring 2
    Stage A, B;
    A.full = in && (kind == 0 || kind == 1);
    A.needU = in && (kind <= 2) && kind >= 0;
    A.needV = in && (kind <= 1 || kind == 3) && kind >= 0;
    A.active = active;
    // stage B: full on the core, partial on ring 1 (u+ on the row above and
    // the right column, v+ on the row below and the left column, p and q on
    // the upper-left and lower-right corners)
    const bool r1_above = kind == 1 && py == y0 + TY && px >= x0 && px < x0 + TX;
    const bool r1_right = kind == 1 && px == x0 + TX && py >= y0 && py < y0 + TY;
    const bool r1_below = kind == 1 && py == y0 - 1 && px >= x0 && px < x0 + TX;
    const bool r1_left = kind == 1 && px == x0 - 1 && py >= y0 && py < y0 + TY;
    const bool r1_ul = kind == 1 && px == x0 - 1 && py == y0 + TY;
    const bool r1_lr = kind == 1 && px == x0 + TX && py == y0 - 1;
    B.full = in && kind == 0;
    B.needU = in && (kind == 0 || r1_above || r1_right);
    B.needV = in && (kind == 0 || r1_below || r1_left);
    B.active = kind == 0 || r1_above || r1_right || r1_below || r1_left || r1_ul || r1_lr;
    // output windows: B writes planes z0..zl; A produces what B reads
    B.z0 = z0;
    B.zl = zl;
    A.z0 = max(z0 - 1, 0);
    A.zl = min(zl + 1, d.nz - 1);
    A.UP1 = A.UB1 = B.UP1 = B.UB1 = 0.0f;
    for (int c = 0; c < 3; c++) A.VB2[c] = B.VB2[c] = 0.0f;

    // memory access: descriptors per field, lane column offset, uniform plane offsets
    const long long col = in ? (long long)px + d.sy * py : 0;
    const int v4 = (int)(col * 4), vS = (int)(col * SB), vH = (int)(col * 16);
    const int comp = (int)(d.n * SB);
    const long long plane4 = d.sz * 4, planeS = d.sz * SB, planeH = d.sz * 16;
    const auto rh = rsrc2(hist, d.n * 16);
    __amdgpu_buffer_rsrc_t ru, rv, rp, rq, wu, wv, wp, wq;
    int fu = 0, fv = 0, fp = 0, fq = 0, gu = 0, gv = 0, gp = 0, gq = 0;  // field offsets (one descriptor)
    if constexpr (UNI) {
        const auto rs = rsrc2(sp.base, sp.bytes);
        ru = rv = rp = rq = wu = wv = wp = wq = rs;
        fu = sp.u0; fv = sp.v0; fp = sp.p0; fq = sp.q0;
        gu = sp.u1; gv = sp.v1; gp = sp.p1; gq = sp.q1;
    } else {
        ru = rsrc2(Xc.u, d.n * 4); rv = rsrc2(Xc.v, 3 * d.n * SB); rp = rsrc2(Yc.p, 3 * d.n * SB);
        rq = rsrc2(Yc.q, 6 * d.n * SB);
        wu = rsrc2(Xn.u, d.n * 4); wv = rsrc2(Xn.v, 3 * d.n * SB); wp = rsrc2(Yn.p, 3 * d.n * SB);
        wq = rsrc2(Yn.q, 6 * d.n * SB);
    }

    auto load_state = [&](Pl &P, uint32_t hw[4], int s, int m) {
        const int sc = s < d.nz ? s : d.nz - 1;
        const int o4 = (int)(plane4 * sc), oS = (int)(planeS * sc), oH = (int)(planeH * sc);
        P.u = Io2<0>::ld(ru, (m & LD2_U) ? v4 : LD2_SKIP, o4 + fu);
        const int ov = (m & LD2_V) ? vS : LD2_SKIP;
        for (int c = 0; c < 3; c++) P.v[c] = Io2<STORE>::ld(rv, ov, fv + oS + c * comp);
        for (int c = 0; c < 3; c++)
            P.p[c] = Io2<STORE>::ld(rp, (m & (LD2_PX << c)) ? vS : LD2_SKIP, fp + oS + c * comp);
        for (int c = 0; c < 6; c++)
            P.q[c] = Io2<STORE>::ld(rq, (m & (LD2_Q0 << c)) ? vS : LD2_SKIP, fq + oS + c * comp);
        auto hv = __builtin_amdgcn_raw_buffer_load_b128(rh, (m & LD2_H) ? vH : LD2_SKIP, oH, 0);
        hw[0] = hv[0];
        hw[1] = hv[1];
        hw[2] = hv[2];
        hw[3] = hv[3];
    };
    // 16-bit storage: the plane's fields are loaded as raw bits into the
    // registers of its slot and converted in place when it becomes the
    // current plane, a step later (converting at the load would wait for it
    // and stall the prefetch; a separate buffer for the bits would need
    // register copies, and a copy of a register whose load is in flight
    // waits for every memory operation of the wave).  u is float32 in every
    // storage and is loaded as it is.
    auto load_raw = [&](Pl &P, uint32_t hw[4], int s, int m) {
        const int sc = s < d.nz ? s : d.nz - 1;
        const int o4 = (int)(plane4 * sc), oS = (int)(planeS * sc), oH = (int)(planeH * sc);
        P.u = Io2<0>::ld(ru, (m & LD2_U) ? v4 : LD2_SKIP, o4);
        const int ov = (m & LD2_V) ? vS : LD2_SKIP;
        for (int c = 0; c < 3; c++) P.v[c] = __uint_as_float(Io2<STORE == 0 ? 1 : STORE>::raw(rv, ov, oS + c * comp));
        for (int c = 0; c < 3; c++)
            P.p[c] = __uint_as_float(
                Io2<STORE == 0 ? 1 : STORE>::raw(rp, (m & (LD2_PX << c)) ? vS : LD2_SKIP, oS + c * comp));
        for (int c = 0; c < 6; c++)
            P.q[c] = __uint_as_float(
                Io2<STORE == 0 ? 1 : STORE>::raw(rq, (m & (LD2_Q0 << c)) ? vS : LD2_SKIP, oS + c * comp));
        auto hv = __builtin_amdgcn_raw_buffer_load_b128(rh, (m & LD2_H) ? vH : LD2_SKIP, oH, 0);
        hw[0] = hv[0];
        hw[1] = hv[1];
        hw[2] = hv[2];
        hw[3] = hv[3];
    };
    auto convert = [&](Pl &P) {
        for (int c = 0; c < 3; c++) P.v[c] = Io2<STORE == 0 ? 1 : STORE>::cvt(__float_as_uint(P.v[c]));
        for (int c = 0; c < 3; c++) P.p[c] = Io2<STORE == 0 ? 1 : STORE>::cvt(__float_as_uint(P.p[c]));
        for (int c = 0; c < 6; c++) P.q[c] = Io2<STORE == 0 ? 1 : STORE>::cvt(__float_as_uint(P.q[c]));
    };

    // phase 1: publish p_x, p_y of plane s (cur) and q of plane s-1 (prev)
    auto publish = [&](L &l, const Stage &S, const Pl &cur, const Pl &prev) {
        if (S.active) {
            l.sPx[e] = cur.p[0];
            l.sPy[e] = cur.p[1];
            l.sQ[0 * NE + e] = prev.q[0];
            l.sQ[1 * NE + e] = prev.q[1];
            l.sQ[2 * NE + e] = prev.q[3];
            l.sQ[3 * NE + e] = prev.q[4];
            l.sQ[4 * NE + e] = prev.q[5];
        }
    };
    // phase 2: u+ at plane s, v+ at plane s-1; publish ubar(s-1), vbar(s-1)
    auto primal = [&](L &l, Stage &S, const Pl &cur, const Pl &prev, const uint32_t hw[4], int s) {
        const int sv = s - 1;
        const bool do_u = s >= S.z0 && s < d.nz;
        const bool do_v = sv >= max(S.z0 - 1, 0) && sv <= S.zl;
        const bool zlo_s = s > 0, zhi_s = s < d.nz - 1, zlo_v = sv > 0, zhi_v = sv < d.nz - 1;
        S.UP = S.UB = 0.0f;
        for (int c = 0; c < 3; c++) S.VP[c] = S.VB[c] = 0.0f;
        if (S.needU && do_u) {
            const bool fz = d.halo > 0 && (s < d.halo || s >= d.nz - d.halo);
            float pm[3];
            const float lx = l.sPx[e - 1], ly = l.sPy[e - EX];
            pm[0] = mlo_x ? lx : 0.0f;
            pm[1] = mlo_y ? ly : 0.0f;
            pm[2] = zlo_s ? prev.p[2] : 0.0f;
            const bool mlo[3] = {mlo_x, mlo_y, zlo_s}, mhi[3] = {mhi_x, mhi_y, zhi_s};
            S.UP = primal_u(cur.u, cur.p, pm, mlo, mhi, fxy || fz, hw, cf);
            S.UB = 2.0f * S.UP - cur.u;
        }
        if (S.needV && do_v) {
            float qn[3][3];
            for (int i = 0; i < 3; i++) {
                const float ax = l.sQ[lq2(qslot(i, 0)) * NE + e + 1];
                const float ay = l.sQ[lq2(qslot(i, 1)) * NE + e + EX];
                qn[i][0] = mhi_x ? ax : 0.0f;
                qn[i][1] = mhi_y ? ay : 0.0f;
                qn[i][2] = zhi_v ? cur.q[qslot(i, 2)] : 0.0f;
            }
            const bool mlo[3] = {mlo_x, mlo_y, zlo_v}, mhi[3] = {mhi_x, mhi_y, zhi_v};
            primal_v(S.VP, prev.v, prev.p, prev.q, qn, mlo, mhi, cf);
            for (int i = 0; i < 3; i++) {
                S.VP[i] = rnd<STORE>(S.VP[i]);
                S.VB[i] = 2.0f * S.VP[i] - prev.v[i];
            }
        }
        if (S.needU) l.sU[e] = S.UB1;
        if (S.needV) {
            l.sV[0 * NE + e] = S.VB[0];
            l.sV[1 * NE + e] = S.VB[1];
            l.sV[2 * NE + e] = S.VB[2];
        }
    };
    // phase 3: dual update of plane s-1 into `out` (u+, v+, p, q of plane s-1);
    // returns whether this column produced a result for that plane.  p and q
    // are rounded to the storage precision where they are computed on
    // (stage A); stage B only stores them, and the store rounds them the
    // same way (rounding is idempotent), so it skips the round trip.
    auto dual = [&](L &l, Stage &S, const Pl &prev, int s, Pl &out, bool round_pq) -> bool {
        const int sv = s - 1;
        const bool do_dual = sv >= S.z0 && sv <= S.zl;
        bool made = false;
        if (S.full && do_dual) {
            const bool zlo_v = sv > 0, zhi_v = sv < d.nz - 1;
            const bool mlo[3] = {mlo_x, mlo_y, zlo_v}, mhi[3] = {mhi_x, mhi_y, zhi_v};
            float ub_hi[3], vb_lo[3][3];
            const float ux = l.sU[e + 1], uy = l.sU[e + EX];
            ub_hi[0] = mhi_x ? ux : 0.0f;
            ub_hi[1] = mhi_y ? uy : 0.0f;
            ub_hi[2] = zhi_v ? S.UB : 0.0f;
            for (int i = 0; i < 3; i++) {
                const float bx = l.sV[i * NE + e - 1], by = l.sV[i * NE + e - EX];
                vb_lo[0][i] = mlo_x ? bx : 0.0f;
                vb_lo[1][i] = mlo_y ? by : 0.0f;
                vb_lo[2][i] = zlo_v ? S.VB2[i] : 0.0f;
            }
            out.u = S.UP1;
            for (int c = 0; c < 3; c++) {
                out.v[c] = S.VP[c];
                out.p[c] = prev.p[c];
            }
            for (int c = 0; c < 6; c++) out.q[c] = prev.q[c];
            dual_pq(out.p, out.q, S.UB1, ub_hi, S.VB, vb_lo, mlo, mhi, cf);
            if (round_pq) {
                for (int c = 0; c < 3; c++) out.p[c] = rnd<STORE>(out.p[c]);
                for (int c = 0; c < 6; c++) out.q[c] = rnd<STORE>(out.q[c]);
            }
            made = true;
        }
        S.UP1 = S.UP;
        S.UB1 = S.UB;
        for (int c = 0; c < 3; c++) S.VB2[c] = S.VB[c];
        return made;
    };

    // Stage A walks planes s = sA0..sA1 with (prev, cur, next) = planes
    // s-1, s, s+1 of the state in memory and produces the full update of
    // plane s-1.  Stage B walks one step later than it could, at plane
    // sb = s - 2, so both stages share the two barriers of a step: its
    // (prev, cur) are stage A's results for planes s-3 and s-2, and the
    // histogram of plane s-2 is kept from stage A's plane s-2.  Both stages
    // keep three plane slots that rotate by one per step; the loop is
    // unrolled three times so the rotation is a renaming, not a copy, and
    // stage A writes its result into the slot stage B has just finished.
    struct PlH {
        Pl f;
        uint32_t h[4];
    };
    PlH a0, a1, a2;
    Pl b0, b1, b2;
    a0.f.u = 0.0f;
    for (int c = 0; c < 3; c++) a0.f.p[c] = a0.f.v[c] = 0.0f;
    for (int c = 0; c < 6; c++) a0.f.q[c] = 0.0f;
    for (int c = 0; c < 4; c++) a0.h[c] = 0u;
    b0 = a0.f;
    b1 = a0.f;
    b2 = a0.f;
    const int sA0 = max(A.z0 - 1, 0), sA1 = A.zl + 1;
    const int sB0 = max(B.z0 - 1, 0), sB1 = B.zl + 1;
    const int s_end = sB1 + 2;
    if (STORE == 0) load_state(a1.f, a1.h, sA0, lmask);
    else load_raw(a1.f, a1.h, sA0, lmask);

    // one plane step: stage A on (prev, cur, next) = (ap, ac, an), stage B on
    // (prev, cur) = (bp, bc), stage A's result into bo
    auto step = [&](PlH &ap, PlH &ac, PlH &an, Pl &bp, Pl &bc, Pl &bo, int s) {
        const bool runA = s <= sA1;
        const int sb = s - 2;
        const bool runB = sb >= sB0;
        if (STORE != 0 && runA) convert(ac.f);
        // phase 1
        if (runA) publish(la, A, ac.f, ap.f);
        if (runB) publish(lb, B, bc, bp);
        // prefetch plane s+1, issued at every step (with every field masked
        // off when stage A needs no further plane): the memory counter then
        // sees the same loads on every path and waits for exactly the plane
        // in use, not for the prefetch in flight
        const int pm = (runA && s + 1 <= sA1) ? lmask : 0;
        if (STORE == 0) load_state(an.f, an.h, s + 1, pm);
        else load_raw(an.f, an.h, s + 1, pm);
        lds_barrier2();
        // phase 2
        if (runA) {
            primal(la, A, ac.f, ap.f, ac.h, s);
            // stage B reads this plane's histogram two steps later
            lh.h[s % 3][threadIdx.x] = make_uint4(ac.h[0], ac.h[1], ac.h[2], ac.h[3]);
        }
        if (runB) {
            const uint4 hv = lh.h[sb % 3][threadIdx.x];
            const uint32_t hB[4] = {hv.x, hv.y, hv.z, hv.w};
            primal(lb, B, bc, bp, hB, sb);
        }
        lds_barrier2();
        // phase 3 (stage B first: its previous plane is dead before stage A's
        // result, which takes its slot two steps later, is formed)
        if (runB) {
            Pl outB;
            if (dual(lb, B, bp, sb, outB, false) && in) {
                const int sv = sb - 1;
                const int o4 = (int)(plane4 * sv), oS = (int)(planeS * sv);
                Io2<0>::st<SCP>(wu, v4, o4 + gu, outB.u);
                if (!TV)
                    for (int c = 0; c < 3; c++) Io2<STORE>::template st<SCP>(wv, vS, gv + oS + c * comp, outB.v[c]);
                for (int c = 0; c < 3; c++) Io2<STORE>::template st<SCP>(wp, vS, gp + oS + c * comp, outB.p[c]);
                if (!TV)
                    for (int c = 0; c < 6; c++) Io2<STORE>::template st<SCP>(wq, vS, gq + oS + c * comp, outB.q[c]);
            }
        }
        if (runA) dual(la, A, ap.f, s, bo, true);
    };
    // No early exit inside the unrolled loop: one or two trailing steps past
    // s_end load and store nothing, and without the exits the values in flight
    // need no copies at the loop's merge points (a copy of a register whose
    // load is in flight waits for every memory operation of the wave).
    if constexpr (STORE == 0) {
        for (int s = sA0; s <= s_end; s += 3) {
            step(a0, a1, a2, b0, b1, b2, s);
            step(a1, a2, a0, b1, b2, b0, s + 1);
            step(a2, a0, a1, b2, b0, b1, s + 2);
        }
    } else {
        // 16-bit storage: the loop runs at least once (s_end > sA0); without
        // the check for no pass the compiler leaves no full memory wait at
        // its head (FP16 568 -> 552 us per launch on 256^3, BF16 565 -> 561;
        // in float32 the same form was 1 % slower)
        int s = sA0;
        do {
            step(a0, a1, a2, b0, b1, b2, s);
            step(a1, a2, a0, b1, b2, b0, s + 1);
            step(a2, a0, a1, b2, b0, b1, s + 2);
            s += 3;
        } while (s <= s_end);
    }
}

template <int STORE, int TY, int SCP, bool TV = false, bool UNI = false>
__global__ void __launch_bounds__(TX *(TY + 5), TILED2_WAVES_PER_EU)
    k_fused2_tiled(XBuf<STORE> Xc, YBuf<STORE> Yc, XBuf<STORE> Xn, YBuf<STORE> Yn, const uint16_t *__restrict__ hist,
                   Dims d, Coef cf, int CZ, int ntx, int nty, int ntz, Span sp) {
    __shared__ XLds<TY> la, lb;
    __shared__ HLds<TY> lh;
    // XCD-aware tile order, as in the one-iteration kernel
    const int nb = ntx * nty * ntz;
    const int per = (nb + 7) / 8;
    const int T = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
    if (T >= nb) return;
    run_tile2<STORE, TY, SCP, TV, UNI>(la, lb, lh, Xc, Yc, Xn, Yn, hist, d, cf, CZ, T % ntx, (T / ntx) % nty,
                                       T / (ntx * nty), sp);
}

// Batched two-iteration pass: every tile of every block advances two
// iterations per launch.  Workgroups pull tiles from the same per-XCD queue
// segments as the one-iteration batched kernel; no workgroup waits on
// another.
template <int STORE, int TY, bool UNI = false>
__global__ void __launch_bounds__(TX *(TY + 5), TILED2_WAVES_PER_EU)
    k_fused2_batch(const BatchBlock *__restrict__ blocks, const int4 *__restrict__ tiles, int ntiles, int *counters,
                   Coef cf, int flip) {
    __shared__ XLds<TY> la, lb;
    __shared__ HLds<TY> lh;
    __shared__ int s_tile;
    const int seg_len = (ntiles + 7) / 8;
    const int home = (int)(blockIdx.x % 8);
    for (int k = 0; k < 8; k++) {
        const int seg = (home + k) & 7;
        const int seg_end = min(seg_len * (seg + 1), ntiles);
        while (true) {
            if (threadIdx.x == 0) s_tile = seg * seg_len + atomicAdd(&counters[seg], 1);
            lds_barrier2();
            const int ti = s_tile;
            lds_barrier2();  // everyone has read s_tile before it is rewritten
            if (ti >= seg_end) break;
            const int4 tr = tiles[ti];
            const BatchBlock &bb = blocks[tr.x];
            const int xc = bb.xc ^ flip, yc = bb.yc ^ flip;
            XBuf<STORE> Xc{bb.u[xc], (typename Store<STORE>::T *)bb.v[xc]};
            XBuf<STORE> Xn{bb.u[xc ^ 1], (typename Store<STORE>::T *)bb.v[xc ^ 1]};
            YBuf<STORE> Yc{(typename Store<STORE>::T *)bb.p[yc], (typename Store<STORE>::T *)bb.q[yc]};
            YBuf<STORE> Yn{(typename Store<STORE>::T *)bb.p[yc ^ 1], (typename Store<STORE>::T *)bb.q[yc ^ 1]};
            if constexpr (UNI) {
                // every field within the state's allocation (below 2 GiB):
                // one descriptor and scalar byte offsets, as in the one-block
                // kernel (the offsets are made wave-uniform explicitly; kept
                // in vector registers they would turn every store into a
                // loop over the distinct offsets)
                const char *base = (const char *)bb.u[0];
                auto off = [&](const void *f) {
                    return __builtin_amdgcn_readfirstlane((int)((const char *)f - base));
                };
                const Span sp{base,          bb.span,           off(bb.u[xc]),     off(bb.v[xc]),     off(bb.p[yc]),
                              off(bb.q[yc]), off(bb.u[xc ^ 1]), off(bb.v[xc ^ 1]), off(bb.p[yc ^ 1]), off(bb.q[yc ^ 1])};
                run_tile2<STORE, TY, 0, false, true>(la, lb, lh, Xc, Yc, Xn, Yn, bb.hist, bb.d, cf, bb.cz,
                                                     tr.y & 0xffff, tr.y >> 16, tr.z, sp);
            } else {
                run_tile2<STORE, TY, 0>(la, lb, lh, Xc, Yc, Xn, Yn, bb.hist, bb.d, cf, bb.cz, tr.y & 0xffff,
                                        tr.y >> 16, tr.z);
            }
            lds_barrier2();  // the tile's LDS reads are done before the next tile writes
        }
    }
}

// the one-descriptor form when every field lies within 2 GiB of the lowest
static bool state_span(const SolveBufs &b, const Dims &d, int sb, Span &sp) {
    const char *f[8] = {(const char *)b.xc_u, (const char *)b.xc_v, (const char *)b.yc_p, (const char *)b.yc_q,
                        (const char *)b.xo_u, (const char *)b.xo_v, (const char *)b.yo_p, (const char *)b.yo_q};
    const long long len[8] = {4 * d.n, 3 * d.n * sb, 3 * d.n * sb, 6 * d.n * sb,
                              4 * d.n, 3 * d.n * sb, 3 * d.n * sb, 6 * d.n * sb};
    const char *lo = f[0];
    const char *hi = f[0] + len[0];
    for (int k = 1; k < 8; k++) {
        lo = f[k] < lo ? f[k] : lo;
        hi = f[k] + len[k] > hi ? f[k] + len[k] : hi;
    }
    if (hi - lo >= (1LL << 31)) return false;
    sp.base = lo;
    sp.bytes = (int)(hi - lo);
    int *o[8] = {&sp.u0, &sp.v0, &sp.p0, &sp.q0, &sp.u1, &sp.v1, &sp.p1, &sp.q1};
    for (int k = 0; k < 8; k++) *o[k] = (int)(f[k] - lo);
    return true;
}

template <int STORE, int TY, int SCP, bool TV = false>
static void launch2_ty(const SolveBufs &b, const Dims &d, const Coef &cf, int cz, hipStream_t s) {
    XBuf<STORE> Xc{b.xc_u, (typename Store<STORE>::T *)b.xc_v};
    XBuf<STORE> Xo{b.xo_u, (typename Store<STORE>::T *)b.xo_v};
    YBuf<STORE> Yc{(typename Store<STORE>::T *)b.yc_p, (typename Store<STORE>::T *)b.yc_q};
    YBuf<STORE> Yo{(typename Store<STORE>::T *)b.yo_p, (typename Store<STORE>::T *)b.yo_q};
    int ntx = (d.nx + TX - 1) / TX, nty = (d.ny + TY - 1) / TY, ntz = (d.nz + cz - 1) / cz;
    int nb = ntx * nty * ntz;
    int per = (nb + 7) / 8;
    Span sp{};
    if (STORE == 0 && TY == 7 && state_span(b, d, 4, sp))
        hipLaunchKernelGGL((k_fused2_tiled<STORE, TY, SCP, TV, (STORE == 0 && TY == 7)>), dim3(8 * per),
                           dim3(TX * (TY + 5)), 0, s, Xc, Yc, Xo, Yo, b.hist, d, cf, cz, ntx, nty, ntz, sp);
    else
        hipLaunchKernelGGL((k_fused2_tiled<STORE, TY, SCP, TV>), dim3(8 * per), dim3(TX * (TY + 5)), 0, s, Xc, Yc, Xo,
                           Yo, b.hist, d, cf, cz, ntx, nty, ntz, sp);
}

template <int STORE, int SCP>
static void launch2_t(const SolveBufs &b, const Dims &d, const Coef &cf, int ty, int cz, hipStream_t s) {
    if (ty == 6) launch2_ty<STORE, 6, SCP>(b, d, cf, cz, s);
    else if (ty == 7 && STORE == 0 && cf.tvl1) launch2_ty<STORE, 7, SCP, true>(b, d, cf, cz, s);
    else if (ty == 7) launch2_ty<STORE, 7, SCP>(b, d, cf, cz, s);
    else launch2_ty<STORE, 4, SCP>(b, d, cf, cz, s);
}

bool tiled2_shape_ok(int ty, int cz) { return (ty == 4 || ty == 6 || ty == 7) && cz >= 1; }

template <int STORE, int TY>
static int batch2_per_cu_t() {
    int nb = 0, nu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_fused2_batch<STORE, TY>, TX * (TY + 5), 0) != hipSuccess)
        return 1;
    // the one-descriptor form shares the grid
    if (STORE == 0 && TY == 7 &&
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&nu, k_fused2_batch<STORE, TY, (STORE == 0 && TY == 7)>,
                                                     TX * (TY + 5), 0) == hipSuccess)
        nb = nu < nb ? nu : nb;
    return nb > 0 ? nb : 1;
}

int batch2_blocks_per_cu(int storage, int ty) {
    if (storage == 0) return ty == 4 ? batch2_per_cu_t<0, 4>() : (ty == 6 ? batch2_per_cu_t<0, 6>() : batch2_per_cu_t<0, 7>());
    if (storage == 1) return ty == 4 ? batch2_per_cu_t<1, 4>() : (ty == 6 ? batch2_per_cu_t<1, 6>() : batch2_per_cu_t<1, 7>());
    return ty == 4 ? batch2_per_cu_t<2, 4>() : (ty == 6 ? batch2_per_cu_t<2, 6>() : batch2_per_cu_t<2, 7>());
}

template <int STORE>
static void launch_batch2_t(const BatchBlock *blocks, const int4 *tiles, int ntiles, int *counters, const Coef &cf,
                            int ty, int flip, int grid, bool span, hipStream_t s) {
    if (STORE == 0 && ty == 7 && span)
        hipLaunchKernelGGL((k_fused2_batch<STORE, 7, (STORE == 0)>), dim3(grid), dim3(TX * 12), 0, s, blocks, tiles,
                           ntiles, counters, cf, flip);
    else if (ty == 4)
        hipLaunchKernelGGL((k_fused2_batch<STORE, 4>), dim3(grid), dim3(TX * 9), 0, s, blocks, tiles, ntiles, counters,
                           cf, flip);
    else if (ty == 6)
        hipLaunchKernelGGL((k_fused2_batch<STORE, 6>), dim3(grid), dim3(TX * 11), 0, s, blocks, tiles, ntiles,
                           counters, cf, flip);
    else
        hipLaunchKernelGGL((k_fused2_batch<STORE, 7>), dim3(grid), dim3(TX * 12), 0, s, blocks, tiles, ntiles,
                           counters, cf, flip);
}

void launch_batch2(int storage, const BatchBlock *blocks, const int4 *tiles, int ntiles, int *counters, const Coef &cf,
                   int ty, int flip, int grid, bool span, hipStream_t s) {
    launch_reset_counters(counters, s);
    if (storage == 0) launch_batch2_t<0>(blocks, tiles, ntiles, counters, cf, ty, flip, grid, span, s);
    else if (storage == 1) launch_batch2_t<1>(blocks, tiles, ntiles, counters, cf, ty, flip, grid, span, s);
    else launch_batch2_t<2>(blocks, tiles, ntiles, counters, cf, ty, flip, grid, span, s);
}

// resident workgroups per CU of the two-iteration kernel
template <int STORE, int TY>
static int per_cu2_t() {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_fused2_tiled<STORE, TY, STORE_CP_STREAM>, TX * (TY + 5),
                                                     0) != hipSuccess)
        return 1;
    return nb > 0 ? nb : 1;
}

template <int STORE>
static int per_cu2_s(int ty) {
    return ty == 4 ? per_cu2_t<STORE, 4>() : (ty == 6 ? per_cu2_t<STORE, 6>() : per_cu2_t<STORE, 7>());
}

int tiled2_blocks_per_cu(int storage, int ty) {
    return storage == 0 ? per_cu2_s<0>(ty) : (storage == 1 ? per_cu2_s<1>(ty) : per_cu2_s<2>(ty));
}

// Planes per z-chunk: a launch runs ceil(tiles / slots) rounds of resident
// workgroups, and a tile of cz planes takes cz + 3 plane steps (the two
// stages' pipeline fill and the z-halo), so the chunk minimising
// rounds x (cz + 3) is taken (ties: the deeper chunk).  On a 256^3 block with
// 64 x 7 tiles and 256 slots this picks 52 planes (740 tiles in three nearly
// full rounds); the model's ratios for 64 and 26 planes (1.22, 1.06) match
// the measured times (1.20, 1.05).  Small blocks get short chunks.
int choose_tile2_z(const Dims &d, int ty, int slots) {
    const long long per_chunk = (long long)((d.nx + TX - 1) / TX) * ((d.ny + ty - 1) / ty);
    const int lo = 1;
    long long best = -1;
    int best_cz = d.nz;
    for (int cz = d.nz; cz >= lo; cz--) {
        const long long tiles = per_chunk * ((d.nz + cz - 1) / cz);
        const long long rounds = (tiles + slots - 1) / slots;
        const long long cost = rounds * (cz + 3);
        if (best < 0 || cost < best) {
            best = cost;
            best_cz = cz;
        }
    }
    return best_cz;
}

void launch_tiled2(int storage, const SolveBufs &b, const Dims &d, const Coef &cf, int ty, int cz, hipStream_t s) {
    if (stream_stores(storage, d)) {
        if (storage == 0) launch2_t<0, STORE_CP_STREAM>(b, d, cf, ty, cz, s);
        else if (storage == 1) launch2_t<1, STORE_CP_STREAM>(b, d, cf, ty, cz, s);
        else launch2_t<2, STORE_CP_STREAM>(b, d, cf, ty, cz, s);
    } else {
        if (storage == 0) launch2_t<0, 0>(b, d, cf, ty, cz, s);
        else if (storage == 1) launch2_t<1, 0>(b, d, cf, ty, cz, s);
        else launch2_t<2, 0>(b, d, cf, ty, cz, s);
    }
}

}  // namespace tgv
