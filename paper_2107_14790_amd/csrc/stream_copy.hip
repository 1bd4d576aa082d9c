// Device-to-device streaming copy: the plain streaming pass (every byte read
// once and written once) that the solver kernels' HBM rates are compared
// against.  Each lane moves UNROLL 16-byte vectors per trip, issuing all
// loads before the first store; NT selects non-temporal loads and stores.
// Workgroups take contiguous runs of the buffer (grid-stride over runs) so
// each XCD streams its own address range.
#include "internal.h"

namespace tgv {

namespace {

constexpr int COPY_THREADS = 256;
typedef float v4f __attribute__((ext_vector_type(4)));

template <int UNROLL, bool NT>
__global__ void __launch_bounds__(COPY_THREADS) k_stream_copy(const v4f *__restrict__ src, v4f *__restrict__ dst,
                                                              long long n4) {
    constexpr long long RUN = (long long)COPY_THREADS * UNROLL;
    const long long runs = n4 / RUN;
    for (long long r = blockIdx.x; r < runs; r += gridDim.x) {
        const long long base = r * RUN + threadIdx.x;
        v4f v[UNROLL];
#pragma unroll
        for (int k = 0; k < UNROLL; k++) {
            if (NT) v[k] = __builtin_nontemporal_load(src + base + k * COPY_THREADS);
            else v[k] = src[base + k * COPY_THREADS];
        }
#pragma unroll
        for (int k = 0; k < UNROLL; k++) {
            if (NT) __builtin_nontemporal_store(v[k], dst + base + k * COPY_THREADS);
            else dst[base + k * COPY_THREADS] = v[k];
        }
    }
    // the tail shorter than one run
    for (long long i = runs * RUN + (long long)blockIdx.x * COPY_THREADS + threadIdx.x; i < n4;
         i += (long long)gridDim.x * COPY_THREADS)
        dst[i] = src[i];
}

template <int UNROLL, bool NT>
void copy_t(const v4f *src, v4f *dst, long long n4, int wg_per_cu, int cus, hipStream_t s) {
    hipLaunchKernelGGL((k_stream_copy<UNROLL, NT>), dim3(cus * wg_per_cu), dim3(COPY_THREADS), 0, s, src, dst, n4);
}

}  // namespace

bool stream_copy_variant_ok(int variant) { return variant >= 0 && variant < 32; }

// variant bits: 0-1 vectors per lane and trip (1, 2, 4, 8), 2 non-temporal,
// 3-4 workgroups per CU in the grid (2, 4, 8, 16)
void launch_stream_copy(const void *src, void *dst, long long n4, int variant, int cus, hipStream_t s) {
    const v4f *a = (const v4f *)src;
    v4f *b = (v4f *)dst;
    const int wg = 2 << ((variant >> 3) & 3);
    switch (variant & 7) {
        case 0: copy_t<1, false>(a, b, n4, wg, cus, s); break;
        case 1: copy_t<2, false>(a, b, n4, wg, cus, s); break;
        case 2: copy_t<4, false>(a, b, n4, wg, cus, s); break;
        case 3: copy_t<8, false>(a, b, n4, wg, cus, s); break;
        case 4: copy_t<1, true>(a, b, n4, wg, cus, s); break;
        case 5: copy_t<2, true>(a, b, n4, wg, cus, s); break;
        case 6: copy_t<4, true>(a, b, n4, wg, cus, s); break;
        default: copy_t<8, true>(a, b, n4, wg, cus, s); break;
    }
}

}  // namespace tgv
