// Internals of libtgv shared by the kernels and the ABI: launch parameters,
// device structs and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/tgv.h"
#include "device_math.h"

namespace tgv {

enum { KIND_DUAL = 0, KIND_PRIMAL = 1, KIND_FUSED = 2 };

// Raw pointers of one solver launch: the current iterate (xc, yc), the
// other buffers (xo, yo) and the histograms.  v/p/q point at storage of
// the state's precision.
struct SolveBufs {
    float *xc_u;
    void *xc_v;
    float *xo_u;
    void *xo_v;
    void *yc_p, *yc_q;
    void *yo_p, *yo_q;
    const uint16_t *hist;
};

// One block of a batched solve as the persistent kernel reads it: the
// state's buffers for both parities and the block's current parities.
// `span`: bytes from u[0] that hold every field of the state when that is
// below 2 GiB (one buffer descriptor serves them all), else 0.
struct BatchBlock {
    float *u[2];
    void *v[2];
    void *p[2];
    void *q[2];
    const uint16_t *hist;
    Dims d;
    int cz;
    int xc, yc;
    int span;
};

// Geometry of a packed pyramid (all cameras the same size).
struct PyrGeom {
    int L;
    int W, H;
    long long cam_stride;
    long long off[24];
    int w[24], h[24];
};

// A camera as the histogram kernel reads it (uniform per loop trip): its
// pose and intrinsics, its own image size and pyramid, and for a 360-degree
// scan the offset of its boundary tables.
struct CamDev {
    float R[9];
    float t[3];
    float fx, fy, cx, cy;
    int vote;
    int model;       // TGV_MODEL_PINHOLE or TGV_MODEL_SCAN360
    int W, H;        // level-0 size
    int L;           // pyramid levels
    int tab;         // scan: float offset of its C, S (W/4 each) and K (H) tables
    long long base;  // float offset of its pyramid in the packed buffer
    int lvl[24];     // float offset of level l from base
};
static_assert(sizeof(CamDev) == 192, "CamDev layout");

// Energy reduction output (device): primal parts (3), dual, nonfinite.
struct EnergyOut {
    double part[3];
    double dual;
    double nonfinite;
};

int64_t storage_bytes(int storage);

void launch_ref(int kind, int storage, const SolveBufs &b, const Dims &d, const Coef &cf, hipStream_t s);

bool tiled_shape_ok(int ty, int cz);
void launch_tiled(int storage, const SolveBufs &b, const Dims &d, const Coef &cf, int ty, int cz, hipStream_t s);
bool tiled_fits(const Dims &d);
// Cache policy of the fused kernels' result stores: non-temporal (buffer
// instruction bit 2 on gfx950) when one iteration moves more than the
// 256 MiB infinity cache holds.  Such a block's results are not read again
// before they would be evicted, and streaming them leaves the L2 to the
// input rows that neighbouring tiles read as their ring (256^3 block: 6 %
// fewer HBM reads, 6 % faster); a smaller block's results are read back
// from the infinity cache by the next iteration, which write-back stores
// allow (city blocks of 36^3..132^3: 16 % faster than streamed).  The
// batched kernel, which also runs small blocks, always uses write-back.
constexpr int STORE_CP_STREAM = 2;
inline bool stream_stores(int storage, const Dims &d) {
    const long long per_voxel = storage == 0 ? 120 : 72;
    return d.n * per_voxel > (256LL << 20);
}

// Default tiles (measured): 64 x 8 x 32 for a float32 block larger than the
// infinity cache (256^3: 5 % faster than 64 x 4), else 64 x 4 x 32 (city
// blocks: 3 % faster than 64 x 8; 16-bit storage at 256^3: 64 x 4 is
// fastest); FUSED2 64 x 7 (twelve waves: one workgroup fills a CU's three
// waves per SIMD) with the chunk depth from choose_tile2_z; the batched
// solve defaults to 64 x 4.
constexpr int DEFAULT_TILE_Z = 32;
constexpr int DEFAULT_BATCH_TILE_Y = 4;
constexpr int DEFAULT_TILE2_Y = 7;
inline int default_tile_y(int storage, const Dims &d) { return (storage == 0 && stream_stores(storage, d)) ? 8 : 4; }
// two fused iterations per launch (temporal blocking), tiles 64 x ty (ty in {4, 6, 7})
bool tiled2_shape_ok(int ty, int cz);
int tiled2_blocks_per_cu(int storage, int ty);
int choose_tile2_z(const Dims &d, int ty, int slots);
int batch_blocks_per_cu(int storage, int ty);
// batched two-iteration pass (tiles 64 x ty, ty in {4, 6, 7}); resets the queue counters first
int batch2_blocks_per_cu(int storage, int ty);
// span: every block's `span` is set (float32 64 x 7 tiles then take the one-descriptor form)
void launch_batch2(int storage, const BatchBlock *blocks, const int4 *tiles, int ntiles, int *counters, const Coef &cf,
                   int ty, int flip, int grid, bool span, hipStream_t s);
void launch_reset_counters(int *counters, hipStream_t s);
int tiled_blocks_per_cu(int storage, int ty, const Dims &d);
int choose_tile_z(const Dims &d, int ty, int slots);
void launch_tiled2(int storage, const SolveBufs &b, const Dims &d, const Coef &cf, int ty, int cz, hipStream_t s);
// one fused iteration of every block listed in `tiles` (int4: block, tix | tiy << 16, tiz, 0)
void launch_batch(int storage, const BatchBlock *blocks, const int4 *tiles, int ntiles, int *counters, const Coef &cf,
                  int ty, int flip, int grid, hipStream_t s);
void launch_energy(int storage, const SolveBufs &b, const Dims &d, const Coef &cf, float lambda, double vbound,
                   double *partials, int nparts, EnergyOut *out, hipStream_t s);
int energy_partials(const Dims &d);
void launch_pyramids(const float *depth, int ncam, const PyrGeom &g, float *pyr, hipStream_t s);
// votes of ncam cameras (tables: the scans' boundary tables); accumulate:
// add to hist's counts instead of overwriting them
void launch_histograms(const float *pyr, const CamDev *cams, int ncam, const float *tables, const tgv_grid &grid,
                       const tgv_bins &bins, bool accumulate, uint16_t *hist, hipStream_t s);
// the scans' boundary tables of a W x H equirectangular map (host)
void scan_tables(int W, int H, float *C, float *S, float *K);
void launch_fill(float *p, float v, long long n, hipStream_t s);
void launch_fill_bytes0(void *p, long long nbytes, hipStream_t s);
void launch_convert(const void *src, int src_storage, void *dst, int dst_storage, long long n, hipStream_t s);

PyrGeom pyr_geom(int W, int H);
bool stream_copy_variant_ok(int variant);
void launch_stream_copy(const void *src, void *dst, long long n4, int variant, int cus, hipStream_t s);
int extract_blocks(const Dims &d);
int extract_runs(const Dims &d);
void launch_prolongate(const float *uc, const Dims &dc, float *uf, const Dims &df, hipStream_t s);
void launch_extract(const float *u, const Dims &d, const tgv_grid &g, unsigned *counts, unsigned long long *offsets,
                    unsigned long long *runs, float4 *pts, long long max_points, hipStream_t s);

}  // namespace tgv
