// Zero-level crossing points of the indicator u on a block (Sec. 4.6: the
// iso-surface points between neighbouring values of different sign, which
// a marching-cubes pass triangulates).  For every grid edge (x, x + e_i)
// whose end values have different signs (u > 0 against u <= 0) the point
//   origin + (x + 1/2 + t e_i) h,  t = u(x) / (u(x) - u(x + e_i)),
// is written as float4 (X, Y, Z, i).  Two passes make the output order
// deterministic (voxel index ascending, then axis): pass 1 counts per
// workgroup, a one-workgroup scan turns counts into offsets, pass 2
// recomputes and writes each point at its rank.
#include "internal.h"

namespace tgv {

constexpr int EXT_THREADS = 256;

// bit i of the result is set when edge (x, x + e_i) changes sign; t[i] is
// its crossing parameter (NaN if an end value is NaN)
__device__ __forceinline__ int crossings_at(const float *__restrict__ u, const Dims &d, long long idx, int x, int y,
                                            int z, float t[3]) {
    const float a = u[idx];
    const bool pa = a > 0.0f;
    int c = 0;
    const int cc[3] = {x, y, z};
    const int nn[3] = {d.nx, d.ny, d.nz};
    const long long st[3] = {1, d.sy, d.sz};
#pragma unroll
    for (int i = 0; i < 3; i++) {
        t[i] = 0.0f;
        if (cc[i] < nn[i] - 1) {
            const float b = u[idx + st[i]];
            if ((b > 0.0f) != pa) {
                t[i] = a / (a - b);
                c |= 1 << i;
            }
        }
    }
    return c;
}

__global__ void __launch_bounds__(EXT_THREADS) k_count_crossings(const float *__restrict__ u, Dims d,
                                                                 unsigned *__restrict__ counts) {
    const long long idx = (long long)blockIdx.x * EXT_THREADS + threadIdx.x;
    int c = 0;
    if (idx < d.n) {
        const int x = (int)(idx % d.nx), y = (int)((idx / d.nx) % d.ny), z = (int)(idx / d.sz);
        float t[3];
        c = __popc(crossings_at(u, d, idx, x, y, z, t));
    }
    __shared__ unsigned s[EXT_THREADS];
    s[threadIdx.x] = c;
    __syncthreads();
    for (int off = EXT_THREADS / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) counts[blockIdx.x] = s[0];
}

// exclusive scan of nblocks counts by one workgroup (sequential chunks of
// EXT_THREADS, each scanned in LDS); offsets[nblocks] = total
__global__ void __launch_bounds__(EXT_THREADS) k_scan_counts(const unsigned *__restrict__ counts, int nblocks,
                                                             unsigned long long *__restrict__ offsets) {
    __shared__ unsigned long long s[EXT_THREADS];
    __shared__ unsigned long long carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int base = 0; base < nblocks; base += EXT_THREADS) {
        const int i = base + threadIdx.x;
        const unsigned long long v = i < nblocks ? counts[i] : 0ull;
        s[threadIdx.x] = v;
        __syncthreads();
        for (int off = 1; off < EXT_THREADS; off <<= 1) {  // inclusive Hillis-Steele scan
            unsigned long long add = threadIdx.x >= off ? s[threadIdx.x - off] : 0ull;
            __syncthreads();
            s[threadIdx.x] += add;
            __syncthreads();
        }
        if (i < nblocks) offsets[i] = carry + s[threadIdx.x] - v;
        __syncthreads();
        if (threadIdx.x == EXT_THREADS - 1) carry += s[EXT_THREADS - 1];
        __syncthreads();
    }
    if (threadIdx.x == 0) offsets[nblocks] = carry;
}

__global__ void __launch_bounds__(EXT_THREADS) k_write_crossings(const float *__restrict__ u, Dims d, tgv_grid g,
                                                                 const unsigned long long *__restrict__ offsets,
                                                                 float4 *__restrict__ pts, long long max_points) {
    const long long idx = (long long)blockIdx.x * EXT_THREADS + threadIdx.x;
    int c = 0, mask = 0, x = 0, y = 0, z = 0;
    float t[3] = {0.0f, 0.0f, 0.0f};
    if (idx < d.n) {
        x = (int)(idx % d.nx);
        y = (int)((idx / d.nx) % d.ny);
        z = (int)(idx / d.sz);
        mask = crossings_at(u, d, idx, x, y, z, t);
        c = __popc(mask);
    }
    __shared__ unsigned s[EXT_THREADS];
    s[threadIdx.x] = c;
    __syncthreads();
    for (int off = 1; off < EXT_THREADS; off <<= 1) {
        unsigned add = threadIdx.x >= off ? s[threadIdx.x - off] : 0u;
        __syncthreads();
        s[threadIdx.x] += add;
        __syncthreads();
    }
    unsigned long long k = offsets[blockIdx.x] + s[threadIdx.x] - c;
    const float cx = g.origin[0] + ((float)x + 0.5f) * g.h;
    const float cy = g.origin[1] + ((float)y + 0.5f) * g.h;
    const float cz = g.origin[2] + ((float)z + 0.5f) * g.h;
#pragma unroll
    for (int i = 0; i < 3; i++) {
        if (mask & (1 << i)) {
            if ((long long)k < max_points) {
                float4 p = make_float4(cx, cy, cz, (float)i);
                if (i == 0) p.x = cx + t[i] * g.h;
                else if (i == 1) p.y = cy + t[i] * g.h;
                else p.z = cz + t[i] * g.h;
                pts[k] = p;
            }
            k++;
        }
    }
}

__global__ void k_prolongate(const float *__restrict__ uc, Dims dc, float *__restrict__ uf, Dims df) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z = blockIdx.z;
    if (x >= df.nx || y >= df.ny) return;
    uf[(long long)x + df.sy * y + df.sz * z] = uc[(long long)(x >> 1) + dc.sy * (y >> 1) + dc.sz * (z >> 1)];
}

void launch_prolongate(const float *uc, const Dims &dc, float *uf, const Dims &df, hipStream_t s) {
    hipLaunchKernelGGL(k_prolongate, dim3((df.nx + 63) / 64, (df.ny + 3) / 4, df.nz), dim3(64, 4, 1), 0, s, uc, dc, uf,
                       df);
}

int extract_blocks(const Dims &d) { return (int)((d.n + EXT_THREADS - 1) / EXT_THREADS); }

void launch_extract(const float *u, const Dims &d, const tgv_grid &g, unsigned *counts, unsigned long long *offsets,
                    float4 *pts, long long max_points, hipStream_t s) {
    const int nb = extract_blocks(d);
    hipLaunchKernelGGL(k_count_crossings, dim3(nb), dim3(EXT_THREADS), 0, s, u, d, counts);
    hipLaunchKernelGGL(k_scan_counts, dim3(1), dim3(EXT_THREADS), 0, s, counts, nb, offsets);
    if (pts && max_points > 0)
        hipLaunchKernelGGL(k_write_crossings, dim3(nb), dim3(EXT_THREADS), 0, s, u, d, g, offsets, pts, max_points);
}

}  // namespace tgv
