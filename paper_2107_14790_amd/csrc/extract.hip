// Zero-level crossing points of the indicator u on a block (Sec. 4.6: the
// iso-surface points between neighbouring values of different sign, which
// a marching-cubes pass triangulates).  For every grid edge (x, x + e_i)
// whose end values have different signs (u > 0 against u <= 0) the point
//   origin + (x + 1/2 + t e_i) h,  t = u(x) / (u(x) - u(x + e_i)),
// is written as float4 (X, Y, Z, i).  Two passes make the output order
// deterministic (voxel index ascending, then axis): pass 1 counts per
// workgroup, a scan turns the counts into offsets (each scan workgroup
// scans 1024 counts, one more workgroup scans their totals), pass 2
// recomputes and writes each point at its rank.
#include "internal.h"

namespace tgv {

constexpr int EXT_THREADS = 256;
constexpr int SCAN_THREADS = 1024;

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

// sum over the wave of c in 0..3 (two ballots), and over the lanes below
// this one
__device__ __forceinline__ unsigned wave_sum(int c, unsigned &below) {
    const unsigned long long b0 = __ballot(c & 1), b1 = __ballot(c & 2);
    const int lane = threadIdx.x & 63;
    const unsigned long long lt = lane ? (~0ull >> (64 - lane)) : 0ull;
    below = (unsigned)(__popcll(b0 & lt) + 2 * __popcll(b1 & lt));
    return (unsigned)(__popcll(b0) + 2 * __popcll(b1));
}

__global__ void __launch_bounds__(EXT_THREADS) k_count_crossings(const float *__restrict__ u, Dims d,
                                                                 unsigned *__restrict__ counts) {
    const long long idx = (long long)blockIdx.x * EXT_THREADS + threadIdx.x;
    int c = 0;
    if (idx < d.n) {
        const unsigned i = (unsigned)idx, nx = (unsigned)d.nx, row = i / nx;
        const int x = (int)(i - row * nx), y = (int)(row % (unsigned)d.ny), z = (int)(row / (unsigned)d.ny);
        float t[3];
        c = __popc(crossings_at(u, d, idx, x, y, z, t));
    }
    __shared__ unsigned ws[EXT_THREADS / 64];
    unsigned below;
    const unsigned w = wave_sum(c, below);
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x / 64] = w;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned tot = 0;
        for (int k = 0; k < EXT_THREADS / 64; k++) tot += ws[k];
        counts[blockIdx.x] = tot;
    }
}

// inclusive scan of one value per thread of a SCAN_THREADS workgroup
__device__ __forceinline__ unsigned long long block_scan(unsigned long long v, unsigned long long *s) {
    s[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < SCAN_THREADS; off <<= 1) {  // Hillis-Steele
        const unsigned long long add = (int)threadIdx.x >= off ? s[threadIdx.x - off] : 0ull;
        __syncthreads();
        s[threadIdx.x] += add;
        __syncthreads();
    }
    return s[threadIdx.x];
}

// offsets within each run of SCAN_THREADS counts, and the runs' totals
__global__ void __launch_bounds__(SCAN_THREADS) k_scan_counts(const unsigned *__restrict__ counts, int nblocks,
                                                              unsigned long long *__restrict__ offsets,
                                                              unsigned long long *__restrict__ totals) {
    __shared__ unsigned long long s[SCAN_THREADS];
    const int i = blockIdx.x * SCAN_THREADS + threadIdx.x;
    const unsigned long long v = i < nblocks ? counts[i] : 0ull;
    const unsigned long long inc = block_scan(v, s);
    if (i < nblocks) offsets[i] = inc - v;
    if (threadIdx.x == SCAN_THREADS - 1) totals[blockIdx.x] = inc;
}

// exclusive scan of the runs' totals in place (one workgroup, chunks of
// SCAN_THREADS); offsets[nblocks] = the number of points
__global__ void __launch_bounds__(SCAN_THREADS) k_scan_totals(unsigned long long *__restrict__ totals, int nruns,
                                                              unsigned long long *__restrict__ offsets, int nblocks) {
    __shared__ unsigned long long s[SCAN_THREADS];
    unsigned long long carry = 0;
    for (int base = 0; base < nruns; base += SCAN_THREADS) {
        const int i = base + threadIdx.x;
        const unsigned long long v = i < nruns ? totals[i] : 0ull;
        const unsigned long long inc = block_scan(v, s);
        if (i < nruns) totals[i] = carry + inc - v;
        carry += s[SCAN_THREADS - 1];
        __syncthreads();  // everyone has read s before the next chunk writes it
    }
    if (threadIdx.x == 0) offsets[nblocks] = carry;
}

__global__ void __launch_bounds__(EXT_THREADS) k_write_crossings(const float *__restrict__ u, Dims d, tgv_grid g,
                                                                 const unsigned long long *__restrict__ offsets,
                                                                 const unsigned long long *__restrict__ run_base,
                                                                 float4 *__restrict__ pts, long long max_points) {
    const long long idx = (long long)blockIdx.x * EXT_THREADS + threadIdx.x;
    int c = 0, mask = 0, x = 0, y = 0, z = 0;
    float t[3] = {0.0f, 0.0f, 0.0f};
    if (idx < d.n) {
        const unsigned i = (unsigned)idx, nx = (unsigned)d.nx, row = i / nx;
        x = (int)(i - row * nx);
        y = (int)(row % (unsigned)d.ny);
        z = (int)(row / (unsigned)d.ny);
        mask = crossings_at(u, d, idx, x, y, z, t);
        c = __popc(mask);
    }
    // rank of this voxel's first point: the points of the lower waves of
    // the workgroup and of the lower lanes of this wave come first
    __shared__ unsigned ws[EXT_THREADS / 64];
    unsigned below;
    const unsigned w = wave_sum(c, below);
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x / 64] = w;
    __syncthreads();
    for (int k = 0; k < (int)(threadIdx.x / 64); k++) below += ws[k];
    unsigned long long k = run_base[blockIdx.x / SCAN_THREADS] + offsets[blockIdx.x] + below;
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
int extract_runs(const Dims &d) { return (extract_blocks(d) + SCAN_THREADS - 1) / SCAN_THREADS; }

void launch_extract(const float *u, const Dims &d, const tgv_grid &g, unsigned *counts, unsigned long long *offsets,
                    unsigned long long *runs, float4 *pts, long long max_points, hipStream_t s) {
    const int nb = extract_blocks(d), nr = extract_runs(d);
    hipLaunchKernelGGL(k_count_crossings, dim3(nb), dim3(EXT_THREADS), 0, s, u, d, counts);
    hipLaunchKernelGGL(k_scan_counts, dim3(nr), dim3(SCAN_THREADS), 0, s, counts, nb, offsets, runs);
    hipLaunchKernelGGL(k_scan_totals, dim3(1), dim3(SCAN_THREADS), 0, s, runs, nr, offsets, nb);
    if (pts && max_points > 0)
        hipLaunchKernelGGL(k_write_crossings, dim3(nb), dim3(EXT_THREADS), 0, s, u, d, g, offsets, runs, pts,
                           max_points);
}

}  // namespace tgv
