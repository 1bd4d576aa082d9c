/*
 * CPU oracle for depth-map fusion by TGV minimisation
 * (Out-of-Core Surface Reconstruction via Global TGV Minimization, 2021).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow reference that
 * the GPU library is checked against.  It shares no code with the GPU
 * library and must never be linked into it; only tests, the smoke check
 * and the benchmark's CPU-baseline leg load it.
 *
 * Two parts:
 *   1. Depth-map pyramids and the per-(voxel, depth map) histogram vote of
 *      Sec. 3.4, Algorithm 1, in canonical IEEE binary32 arithmetic (every
 *      operation rounded separately, no fused multiply-add; build with
 *      -ffp-contract=off), so that integer bin counts are reproducible
 *      bit for bit by any implementation that follows the same order.
 *   2. The TGV-L1 energy of Eq. 2 (with the symmetric gradient of Eq. 3
 *      and the data weight lambda of Eq. 1) on a regular voxel block, and
 *      its minimisation by the first-order primal-dual method the paper
 *      adopts (Sec. 3.2), in float64: dual ascent with projection onto
 *      the norm balls, primal descent with the proximal map of the
 *      histogram data term, over-relaxation with theta = 1.  Voxels in a
 *      border layer of width `halo` keep u frozen (Sec. 4.5, Fig. 7).
 *
 * Discretisation (the paper does not print one; these are the readings
 * the oracle fixes, all in voxel units):
 *   (grad u)_i(x) = u(x+e_i) - u(x)  where x_i < n_i - 1, dropped (0) else;
 *   d-_j w(x)     = w(x) - w(x-e_j)  where x_j > 0, 0 else;
 *   E(v)_ii = d-_i v_i,  E(v)_ij = (d-_j v_i + d-_i v_j) / 2  (i != j);
 *   K(u, v) = (M.(grad u - v), E v), M_i(x) = [x_i < n_i - 1];
 *   |p| Euclidean; |q|^2 = q_xx^2 + q_yy^2 + q_zz^2 + 2 (q_xy^2 + q_xz^2 + q_yz^2),
 *   the norm of the symmetric matrix, with the matching inner product.
 * Layout: voxel index x + nx*(y + ny*z); vector fields are component-major
 * (v[c*n + idx]); q components ordered xx, yy, zz, xy, xz, yz.
 *
 * Threads: single-threaded unless or_set_threads asks for more.  Only the
 * per-voxel loops of the histogram vote and of the two sweeps of an
 * iteration (all of which write one voxel's own entries from inputs no
 * voxel of the same loop writes) are split over threads, so every result
 * is bit for bit the same at any thread count; sums stay serial.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

static int g_threads = 1;

/* number of threads of the per-voxel loops (1 = the plain serial oracle) */
void or_set_threads(int k) { g_threads = k > 0 ? k : 1; }
int or_get_threads(void) { return g_threads; }

/* ======================================================================
 * Part 1: pyramids and histogram votes (canonical binary32)
 * ====================================================================== */

/* Level l+1 of a pyramid halves each side, rounding up, so that every
 * pixel of level l has exactly one parent; the last level is 1 x 1. */
int or_pyr_levels(int W, int H)
{
    int L = 1;
    while (W > 1 || H > 1) {
        W = (W + 1) >> 1;
        H = (H + 1) >> 1;
        L++;
    }
    return L;
}

long or_pyr_floats(int W, int H)
{
    long total = (long)W * H;
    while (W > 1 || H > 1) {
        W = (W + 1) >> 1;
        H = (H + 1) >> 1;
        total += (long)W * H;
    }
    return total;
}

/* A depth sample is usable when it is finite and positive (Alg. 1 treats
 * anything else as "no ray in this direction"). */
static float canonical_depth(float d)
{
    return (isfinite(d) && d > 0.0f) ? d : 0.0f;
}

/* Mipmap pyramid of one depth map (Sec. 3.4: depth maps are turned into
 * mipmaps so that a voxel larger than a pixel reads a matching level of
 * detail).  A level-(l+1) pixel is the mean of its valid children, taken
 * in the order (2i,2j), (2i+1,2j), (2i,2j+1), (2i+1,2j+1), summed left to
 * right in binary32 and divided by the count; 0 when no child is valid. */
void or_pyramid(const float *depth, int W, int H, float *pyr)
{
    for (long k = 0; k < (long)W * H; k++)
        pyr[k] = canonical_depth(depth[k]);
    const float *src = pyr;
    float *dst = pyr + (long)W * H;
    int w = W, h = H;
    while (w > 1 || h > 1) {
        int w2 = (w + 1) >> 1, h2 = (h + 1) >> 1;
        for (int j = 0; j < h2; j++) {
            for (int i = 0; i < w2; i++) {
                float sum = 0.0f;
                int cnt = 0;
                int cx[4] = {2 * i, 2 * i + 1, 2 * i, 2 * i + 1};
                int cy[4] = {2 * j, 2 * j, 2 * j + 1, 2 * j + 1};
                for (int c = 0; c < 4; c++) {
                    if (cx[c] >= w || cy[c] >= h) continue;
                    float d = src[(long)cy[c] * w + cx[c]];
                    if (d > 0.0f) {
                        sum = sum + d;
                        cnt++;
                    }
                }
                dst[(long)j * w2 + i] = cnt ? sum / (float)cnt : 0.0f;
            }
        }
        src = dst;
        dst += (long)w2 * h2;
        w = w2;
        h = h2;
    }
}

/* Boundary tables of an equirectangular 360-degree scan of W x H pixels
 * (W a multiple of 4).  Column c covers the azimuths [2 pi c / W,
 * 2 pi (c + 1) / W) measured in the scanner's x-y plane from +x towards
 * +y; row r covers the polar angles [pi r / H, pi (r + 1) / H) measured
 * from +z.  The boundary directions, rounded to binary32 from float64:
 *   C[i] = cos(2 pi i / W), S[i] = sin(2 pi i / W)   for i in [0, W/4)
 *   (the column boundaries of one quadrant; the others are these turned
 *   by multiples of 90 degrees),
 *   K[j] = cos(pi j / H)                              for j in [0, H). */
void or_scan_tables(int W, int H, float *C, float *S, float *K)
{
    for (int i = 0; i < W / 4; i++) {
        double a = (6.283185307179586 * (double)i) / (double)W;
        C[i] = (float)cos(a);
        S[i] = (float)sin(a);
    }
    for (int j = 0; j < H; j++) {
        double a = (3.141592653589793 * (double)j) / (double)H;
        K[j] = (float)cos(a);
    }
}

/* Pixel of the direction (x, y, z) (scanner frame, binary32) of length
 * rho in an equirectangular scan, decided by sign tests only:
 *   quadrant q of (x, y): 0 if x > 0, y >= 0; 1 if x <= 0, y > 0;
 *   2 if x < 0, y <= 0; 3 if x >= 0, y < 0 (the scanner's axis x = y = 0
 *   counts as quadrant 0); (x', y') = (x, y) turned by -90 q degrees
 *   (exact: swaps and negations), so x' >= 0 and y' >= 0;
 *   column = q W/4 + the number of i in [1, W/4) with
 *            fl(fl(C[i] y') - fl(S[i] x')) >= 0 (boundary i at or before
 *            the direction);
 *   row    = the number of j in [1, H) with z <= fl(K[j] rho) (boundary j
 *            at or above the direction).
 * Counted here by brute force over every boundary. */
void or_scan_pixel(float x, float y, float z, float rho, int W, int H, const float *C, const float *S,
                   const float *K, int *col, int *row)
{
    int q;
    float xp, yp;
    if (x > 0.0f && y >= 0.0f) { q = 0; xp = x; yp = y; }
    else if (x <= 0.0f && y > 0.0f) { q = 1; xp = y; yp = -x; }
    else if (x < 0.0f && y <= 0.0f) { q = 2; xp = -x; yp = -y; }
    else if (x >= 0.0f && y < 0.0f) { q = 3; xp = -y; yp = x; }
    else { q = 0; xp = x; yp = y; } /* x = y = 0 */
    int c = 0;
    for (int i = 1; i < W / 4; i++) {
        float a = C[i] * yp;
        float b = S[i] * xp;
        if (a - b >= 0.0f) c++;
    }
    int r = 0;
    for (int j = 1; j < H; j++) {
        float k = K[j] * rho;
        if (z <= k) r++;
    }
    *col = q * (W / 4) + c;
    *row = r;
}

/* Bin of one (voxel, depth map) pair per Algorithm 1, or -1 for no vote.
 *   X = origin + (index + 1/2) h; Xc = R X + t (row by row, left to right);
 *   model 0 (pinhole map of camera-frame z):
 *     no vote if the camera depth z <= 0 or the projection leaves the image
 *     (Alg. 1: the map has no ray in that direction); the voxel's distance
 *     is z and its projected diameter s = h fx / z;
 *   model 1 (equirectangular 360-degree scan of ranges; tab = its C, S, K
 *     tables, see or_scan_tables):
 *     the distance is the range rho = sqrt((x^2 + y^2) + z^2) of Xc (no
 *     vote if 0), the pixel is or_scan_pixel's, and s = h fx / rho with fx
 *     the map's pixels per radian;
 *   s picks level l = floor(log2 s) (clamped to the pyramid), computed
 *   exactly by ilogbf; the pixel at level l is floor(px / 2^l), clamped to
 *   the level size;
 *   a = depth - distance;
 *   no vote if the depth is invalid or a < -eta (occluded region);
 *   a is clamped to [-1, 1] after division by delta and binned:
 *     rule 0: nearest of nbins centres spread evenly over [-1, 1];
 *     rule 1: floor(((a + 1) / 2) * nbins), the paper's floor rule, with
 *             a = +1 folded into the last bin. */
int or_vote_bin(const float *pyr, int W, int H, const float *R, const float *t, const float *intr,
                const float *origin, float h, int i, int j, int k, float delta, float eta_over_delta,
                int nbins, int rule, int model, const float *tab)
{
    float X = origin[0] + ((float)i + 0.5f) * h;
    float Y = origin[1] + ((float)j + 0.5f) * h;
    float Z = origin[2] + ((float)k + 0.5f) * h;
    float xc[3];
    for (int r = 0; r < 3; r++) {
        float acc = R[3 * r + 0] * X;
        acc = acc + R[3 * r + 1] * Y;
        acc = acc + R[3 * r + 2] * Z;
        xc[r] = acc + t[r];
    }
    float fx = intr[0], fy = intr[1], cx = intr[2], cy = intr[3];
    float dist, px, py;
    if (model == 0) {
        float z = xc[2];
        if (!(z > 0.0f)) return -1;
        px = fx * (xc[0] / z) + cx;
        py = fy * (xc[1] / z) + cy;
        if (!(px >= 0.0f && px < (float)W && py >= 0.0f && py < (float)H)) return -1;
        dist = z;
    } else {
        float r2 = xc[0] * xc[0];
        r2 = r2 + xc[1] * xc[1];
        r2 = r2 + xc[2] * xc[2];
        float rho = sqrtf(r2);
        if (!(rho > 0.0f)) return -1;
        int col, row;
        or_scan_pixel(xc[0], xc[1], xc[2], rho, W, H, tab, tab + W / 4, tab + W / 2, &col, &row);
        px = (float)col;
        py = (float)row;
        dist = rho;
    }

    int L = or_pyr_levels(W, H);
    float s = (h * fx) / dist;
    int l = 0;
    if (s >= 1.0f) {
        l = ilogbf(s);
        if (l > L - 1) l = L - 1;
    }
    /* walk to level l */
    const float *lev = pyr;
    int w = W, hh = H;
    for (int m = 0; m < l; m++) {
        lev += (long)w * hh;
        w = (w + 1) >> 1;
        hh = (hh + 1) >> 1;
    }
    int ix = (int)floorf(ldexpf(px, -l));
    int iy = (int)floorf(ldexpf(py, -l));
    if (ix > w - 1) ix = w - 1;
    if (iy > hh - 1) iy = hh - 1;
    float d = lev[(long)iy * w + ix];
    if (d == 0.0f) return -1;

    float a = d - dist;
    float eta = eta_over_delta * delta;
    if (a < -eta) return -1;
    float an = fminf(1.0f, fmaxf(-1.0f, a / delta));
    int bin;
    if (rule == 0) {
        float half = (float)(nbins - 1) / 2.0f;
        bin = (int)floorf((an + 1.0f) * half + 0.5f);
    } else {
        bin = (int)floorf(((an + 1.0f) / 2.0f) * (float)nbins);
    }
    if (bin < 0) bin = 0;
    if (bin > nbins - 1) bin = nbins - 1;
    return bin;
}

/* Histograms of a list of voxels (all voxels when vox == NULL): every
 * depth map votes into each voxel per or_vote_bin, with its own weight
 * (1 for stereo depth maps, larger for near noise-free LIDAR, Alg. 1),
 * its own size wh and model (0 pinhole, 1 equirectangular scan).
 * pyrs holds the pyramids of all cameras back to back; hist is
 * [count][8] uint16, slots >= nbins stay 0.  Returns the largest total
 * vote seen in one voxel (so the caller can detect 16-bit overflow). */
long or_histograms(const float *pyrs, int ncam, const float *R, const float *t, const float *intr,
                   const int32_t *wh, const int32_t *vote, const int32_t *model, const float *origin, float h,
                   int nx, int ny, int nz, float delta, float eta_over_delta, int nbins, int rule,
                   const int64_t *vox, long nvox, uint16_t *hist)
{
    long *off = (long *)malloc(sizeof(long) * (ncam + 1));
    float **tab = (float **)calloc(ncam > 0 ? ncam : 1, sizeof(float *));
    off[0] = 0;
    for (int c = 0; c < ncam; c++) {
        off[c + 1] = off[c] + or_pyr_floats(wh[2 * c], wh[2 * c + 1]);
        if (model[c] == 1) {
            int W = wh[2 * c], H = wh[2 * c + 1];
            tab[c] = (float *)malloc(sizeof(float) * (W / 2 + H));
            or_scan_tables(W, H, tab[c], tab[c] + W / 4, tab[c] + W / 2);
        }
    }
    long count = vox ? nvox : (long)nx * ny * nz;
    long maxtot = 0;
#pragma omp parallel for schedule(dynamic, 256) num_threads(g_threads) reduction(max : maxtot)
    for (long m = 0; m < count; m++) {
        long idx = vox ? (long)vox[m] : m;
        int i = (int)(idx % nx), j = (int)((idx / nx) % ny), k = (int)(idx / ((long)nx * ny));
        long acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        long tot = 0;
        for (int c = 0; c < ncam; c++) {
            int b = or_vote_bin(pyrs + off[c], wh[2 * c], wh[2 * c + 1], R + 9 * c, t + 3 * c, intr + 4 * c,
                                origin, h, i, j, k, delta, eta_over_delta, nbins, rule, model[c], tab[c]);
            if (b >= 0) {
                acc[b] += vote[c];
                tot += vote[c];
            }
        }
        if (tot > maxtot) maxtot = tot;
        for (int b = 0; b < 8; b++) hist[8 * m + b] = (uint16_t)(acc[b] > 65535 ? 65535 : acc[b]);
    }
    for (int c = 0; c < ncam; c++) free(tab[c]);
    free(tab);
    free(off);
    return maxtot;
}

/* ======================================================================
 * Part 2: TGV-L1 energy and its primal-dual minimisation (float64)
 * ====================================================================== */

typedef struct {
    long nx, ny, nz, n;
} dims_t;

static dims_t mkdims(int nx, int ny, int nz)
{
    dims_t d = {nx, ny, nz, (long)nx * ny * nz};
    return d;
}

/* strides of the three axes */
static void strides(dims_t d, long st[3]) { st[0] = 1; st[1] = d.nx; st[2] = d.nx * d.ny; }

static void coords(dims_t d, long idx, long c[3])
{
    c[0] = idx % d.nx;
    c[1] = (idx / d.nx) % d.ny;
    c[2] = idx / (d.nx * d.ny);
}

/* index of q component (i, j) in the xx, yy, zz, xy, xz, yz order */
static int qslot(int i, int j)
{
    if (i == j) return i;
    int a = i < j ? i : j, b = i < j ? j : i;
    if (a == 0 && b == 1) return 3;
    if (a == 0 && b == 2) return 4;
    return 5;
}

/* K(u, v) = (M.(grad u - v), E v): kp[3n], kq[6n] (Eq. 2 and Eq. 3). */
void or_apply_K(int nx, int ny, int nz, const double *u, const double *v, double *kp, double *kq)
{
    dims_t d = mkdims(nx, ny, nz);
    long st[3];
    strides(d, st);
    long nn[3] = {d.nx, d.ny, d.nz};
#pragma omp parallel for schedule(static) num_threads(g_threads)
    for (long x = 0; x < d.n; x++) {
        long c[3];
        coords(d, x, c);
        for (int i = 0; i < 3; i++) {
            int m = c[i] < nn[i] - 1;
            kp[i * d.n + x] = m ? (u[x + st[i]] - u[x]) - v[i * d.n + x] : 0.0;
        }
        /* backward differences of v */
        double dm[3][3]; /* dm[i][j] = d-_j v_i */
        for (int i = 0; i < 3; i++)
            for (int j = 0; j < 3; j++)
                dm[i][j] = c[j] > 0 ? v[i * d.n + x] - v[i * d.n + x - st[j]] : 0.0;
        for (int i = 0; i < 3; i++) kq[i * d.n + x] = dm[i][i];
        kq[3 * d.n + x] = 0.5 * (dm[0][1] + dm[1][0]);
        kq[4 * d.n + x] = 0.5 * (dm[0][2] + dm[2][0]);
        kq[5 * d.n + x] = 0.5 * (dm[1][2] + dm[2][1]);
    }
}

/* K^T(p, q) with the weighted inner product on q: returns
 * gu = grad^T(M.p) = -div p and gv = -M.p + E^T q = -(M.p + div2 q). */
void or_apply_KT(int nx, int ny, int nz, const double *p, const double *q, double *gu, double *gv)
{
    dims_t d = mkdims(nx, ny, nz);
    long st[3];
    strides(d, st);
    long nn[3] = {d.nx, d.ny, d.nz};
#pragma omp parallel for schedule(static) num_threads(g_threads)
    for (long x = 0; x < d.n; x++) {
        long c[3];
        coords(d, x, c);
        /* <grad u, M.p> collects, for u(x): -M_i(x) p_i(x) + M_i(x-e_i) p_i(x-e_i) */
        double acc = 0.0;
        for (int i = 0; i < 3; i++) {
            if (c[i] < nn[i] - 1) acc -= p[i * d.n + x];
            if (c[i] > 0) acc += p[i * d.n + x - st[i]];
        }
        gu[x] = acc;
        /* -M.p plus E^T q: <E v, q> = sum_x sum_ij (d-_j v_i)(x) q_ij(x), so the
         * coefficient of v_i(x) is sum_j ([x_j > 0] q_ij(x) - [x_j < n_j-1] q_ij(x+e_j)) */
        for (int i = 0; i < 3; i++) {
            double g = (c[i] < nn[i] - 1) ? -p[i * d.n + x] : 0.0;
            for (int j = 0; j < 3; j++) {
                int s = qslot(i, j);
                if (c[j] > 0) g += q[s * d.n + x];
                if (c[j] < nn[j] - 1) g -= q[s * d.n + x + st[j]];
            }
            gv[i * d.n + x] = g;
        }
    }
}

/* weighted inner product on q-type fields */
static double qnorm2(const double *q, long n, long x)
{
    return q[x] * q[x] + q[n + x] * q[n + x] + q[2 * n + x] * q[2 * n + x] +
           2.0 * (q[3 * n + x] * q[3 * n + x] + q[4 * n + x] * q[4 * n + x] + q[5 * n + x] * q[5 * n + x]);
}

static int is_frozen(dims_t d, long x, int halo)
{
    if (halo <= 0) return 0;
    long c[3];
    coords(d, x, c);
    long nn[3] = {d.nx, d.ny, d.nz};
    for (int i = 0; i < 3; i++)
        if (c[i] < halo || c[i] >= nn[i] - halo) return 1;
    return 0;
}

/* Objective of the proximal step at w: (w - ut)^2 / (2 tau) + lambda sum_k h_k |w - c_k|. */
static double prox_objective(double w, double ut, const double *hk, const double *ck, int nbins, double tau,
                             double lambda)
{
    double s = 0.0;
    for (int k = 0; k < nbins; k++) s += hk[k] * fabs(w - ck[k]);
    return (w - ut) * (w - ut) / (2.0 * tau) + lambda * s;
}

/* Proximal map of the histogram data term (Eq. 1 data term with the
 * per-voxel histogram replacing the individual distance fields, Sec. 3.4):
 *   argmin_w (w - ut)^2 / (2 tau) + lambda sum_k h_k |w - c_k|,
 * centres ascending.  Found by walking the pieces of the piecewise-linear
 * term: on the open interval between consecutive centres the optimality
 * condition is linear and gives w = ut - tau lambda (2 S_below - W); at a
 * centre c_k the subgradient contains 0 when
 *   ut - tau lambda (2 S_{<=k} - W) <= c_k <= ut - tau lambda (2 S_{<k} - W). */
double or_prox(double ut, const double *hk, const double *ck, int nbins, double tau, double lambda)
{
    double W = 0.0;
    for (int k = 0; k < nbins; k++) W += hk[k];
    double tl = tau * lambda;
    double S = 0.0;
    for (int k = 0; k <= nbins; k++) {
        double lo = k > 0 ? ck[k - 1] : -INFINITY;
        double hi = k < nbins ? ck[k] : INFINITY;
        double w = ut - tl * (2.0 * S - W);
        if (w > lo && w < hi) return w;
        if (k < nbins) {
            double Sk = S + hk[k];
            if (ut - tl * (2.0 * Sk - W) <= ck[k] && ck[k] <= w) return ck[k];
            S = Sk;
        }
    }
    /* rounding left every test false: take the best candidate */
    double best = ut, bestv = INFINITY;
    S = 0.0;
    for (int k = 0; k <= nbins; k++) {
        double cand[2];
        int nc = 0;
        cand[nc++] = ut - tl * (2.0 * S - W);
        if (k < nbins) cand[nc++] = ck[k];
        for (int m = 0; m < nc; m++) {
            double f = prox_objective(cand[m], ut, hk, ck, nbins, tau, lambda);
            if (f < bestv) { bestv = f; best = cand[m]; }
        }
        if (k < nbins) S += hk[k];
    }
    return best;
}

/* Projection onto {|y| <= alpha}: y / max(1, |y| / alpha); alpha = 0 gives 0. */
static void project(double *y[], int m, const double *wts, long x, double alpha)
{
    double n2 = 0.0;
    for (int c = 0; c < m; c++) n2 += wts[c] * y[c][x] * y[c][x];
    double nrm = sqrt(n2);
    if (alpha <= 0.0) {
        for (int c = 0; c < m; c++) y[c][x] = 0.0;
        return;
    }
    double s = nrm / alpha;
    if (s > 1.0)
        for (int c = 0; c < m; c++) y[c][x] /= s;
}

/* With tvl1 set the TV-L1 model of Eq. 1 is solved instead: the same
 * iteration with v held at 0 and no q (K reduces to M.grad); v, vbar and q
 * are set to 0 first, whatever the state held.
 *
 * Primal-dual iterations (first-order primal-dual method with
 * over-relaxation theta = 1) on the saddle-point form of Eq. 2:
 *   p <- P_{alpha1}(p + sigma K_p(ubar, vbar)),  q <- P_{alpha0}(q + sigma K_q(ubar, vbar));
 *   (gu, gv) = K^T(p, q);
 *   u+ = prox(u - tau gu) on free voxels, u+ = u on frozen ones (Fig. 7);
 *   v+ = v - tau gv;
 *   ubar = 2 u+ - u,  vbar = 2 v+ - v.
 * All state arrays are read and written in place; a fresh start passes
 * u = ubar = initial u, v = vbar = p = q = 0. */
void or_solve(int nx, int ny, int nz, int halo, const uint16_t *hist, int nbins, const double *centers,
              double alpha0, double alpha1, double lambda, double tau, double sigma, int iters, double *u,
              double *v, double *p, double *q, double *ubar, double *vbar, int tvl1)
{
    dims_t d = mkdims(nx, ny, nz);
    long n = d.n;
    double *kp = (double *)malloc(sizeof(double) * 3 * n);
    double *kq = (double *)malloc(sizeof(double) * 6 * n);
    double *gu = (double *)malloc(sizeof(double) * n);
    double *gv = (double *)malloc(sizeof(double) * 3 * n);
    const double w3[3] = {1.0, 1.0, 1.0};
    const double w6[6] = {1.0, 1.0, 1.0, 2.0, 2.0, 2.0};
    if (tvl1) { /* Eq. 1 has no v and no q */
        memset(v, 0, sizeof(double) * 3 * n);
        memset(vbar, 0, sizeof(double) * 3 * n);
        memset(q, 0, sizeof(double) * 6 * n);
    }
    for (int it = 0; it < iters; it++) {
        /* dual ascent */
        or_apply_K(nx, ny, nz, ubar, vbar, kp, kq);
#pragma omp parallel for schedule(static) num_threads(g_threads)
        for (long x = 0; x < n; x++) {
            double *pp[3] = {p, p + n, p + 2 * n};
            for (int c = 0; c < 3; c++) p[c * n + x] += sigma * kp[c * n + x];
            project(pp, 3, w3, x, alpha1);
            if (tvl1) continue; /* TV-L1 (Eq. 1): no second-order dual */
            double *qq[6] = {q, q + n, q + 2 * n, q + 3 * n, q + 4 * n, q + 5 * n};
            for (int c = 0; c < 6; c++) q[c * n + x] += sigma * kq[c * n + x];
            project(qq, 6, w6, x, alpha0);
        }
        /* primal descent */
        or_apply_KT(nx, ny, nz, p, q, gu, gv);
#pragma omp parallel for schedule(static) num_threads(g_threads)
        for (long x = 0; x < n; x++) {
            double un;
            if (is_frozen(d, x, halo)) {
                un = u[x];
            } else {
                double hk[8];
                for (int k = 0; k < nbins; k++) hk[k] = (double)hist[8 * x + k];
                un = or_prox(u[x] - tau * gu[x], hk, centers, nbins, tau, lambda);
            }
            ubar[x] = 2.0 * un - u[x];
            u[x] = un;
            if (tvl1) continue; /* TV-L1: v stays 0 */
            for (int c = 0; c < 3; c++) {
                double vn = v[c * n + x] - tau * gv[c * n + x];
                vbar[c * n + x] = 2.0 * vn - v[c * n + x];
                v[c * n + x] = vn;
            }
        }
    }
    free(kp);
    free(kq);
    free(gu);
    free(gv);
}

/* Data term sum_k h_k |w - c_k| of one voxel */
static double data_term(double w, const uint16_t *h8, const double *ck, int nbins)
{
    double s = 0.0;
    for (int k = 0; k < nbins; k++) s += (double)h8[k] * fabs(w - ck[k]);
    return s;
}

/* Discrete Eq. 2: out[0] = alpha1 sum |M.(grad u - v)|, out[1] = alpha0 sum |E v|,
 * out[2] = lambda sum over free voxels of the histogram data term; returns the sum. */
double or_primal_energy(int nx, int ny, int nz, int halo, const uint16_t *hist, int nbins, const double *centers,
                        double alpha0, double alpha1, double lambda, const double *u, const double *v,
                        double *out3)
{
    dims_t d = mkdims(nx, ny, nz);
    long n = d.n;
    double *kp = (double *)malloc(sizeof(double) * 3 * n);
    double *kq = (double *)malloc(sizeof(double) * 6 * n);
    or_apply_K(nx, ny, nz, u, v, kp, kq);
    double e1 = 0.0, e0 = 0.0, ed = 0.0;
    for (long x = 0; x < n; x++) {
        e1 += sqrt(kp[x] * kp[x] + kp[n + x] * kp[n + x] + kp[2 * n + x] * kp[2 * n + x]);
        e0 += sqrt(qnorm2(kq, n, x));
        if (!is_frozen(d, x, halo)) ed += data_term(u[x], hist + 8 * x, centers, nbins);
    }
    free(kp);
    free(kq);
    double r[3] = {alpha1 * e1, alpha0 * e0, lambda * ed};
    if (out3) memcpy(out3, r, sizeof(r));
    return r[0] + r[1] + r[2];
}

/* Dual function of the box-restricted problem (u in [-1, 1] on free
 * voxels, |v(x)| <= vbound): for feasible (p, q)
 *   D = sum_free min_{w in [-1,1]} [w gu(x) + lambda data(w)] + sum_frozen u(x) gu(x)
 *       - vbound sum_x |gv(x)|,   (gu, gv) = K^T(p, q).
 * The inner minimum of a convex piecewise-linear function is attained at
 * a breakpoint or an end, so it is exact over {-1, 1, c_k in [-1, 1]}.
 * D is a lower bound of Eq. 2 over the box (weak duality).  For the TV-L1
 * model (tvl1 set) v is not a variable and its term is absent. */
double or_dual_energy(int nx, int ny, int nz, int halo, const uint16_t *hist, int nbins, const double *centers,
                      double lambda, double vbound, const double *u, const double *p, const double *q, int tvl1)
{
    dims_t d = mkdims(nx, ny, nz);
    long n = d.n;
    double *gu = (double *)malloc(sizeof(double) * n);
    double *gv = (double *)malloc(sizeof(double) * 3 * n);
    or_apply_KT(nx, ny, nz, p, q, gu, gv);
    double D = 0.0;
    for (long x = 0; x < n; x++) {
        if (is_frozen(d, x, halo)) {
            D += u[x] * gu[x];
        } else {
            double best = INFINITY;
            double cand[10];
            int nc = 0;
            cand[nc++] = -1.0;
            cand[nc++] = 1.0;
            for (int k = 0; k < nbins; k++)
                if (centers[k] >= -1.0 && centers[k] <= 1.0) cand[nc++] = centers[k];
            for (int m = 0; m < nc; m++) {
                double f = cand[m] * gu[x] + lambda * data_term(cand[m], hist + 8 * x, centers, nbins);
                if (f < best) best = f;
            }
            D += best;
        }
        if (!tvl1) D -= vbound * sqrt(gv[x] * gv[x] + gv[n + x] * gv[n + x] + gv[2 * n + x] * gv[2 * n + x]);
    }
    free(gu);
    free(gv);
    return D;
}

/* Power iteration for ||K||^2 (largest eigenvalue of K^T K) from a seeded
 * start vector; the primal-dual method converges for tau sigma ||K||^2 < 1. */
double or_norm_K2(int nx, int ny, int nz, int iters, uint64_t seed)
{
    dims_t d = mkdims(nx, ny, nz);
    long n = d.n;
    double *u = (double *)malloc(sizeof(double) * n);
    double *v = (double *)malloc(sizeof(double) * 3 * n);
    double *kp = (double *)malloc(sizeof(double) * 3 * n);
    double *kq = (double *)malloc(sizeof(double) * 6 * n);
    uint64_t s = seed * 6364136223846793005ULL + 1442695040888963407ULL;
    for (long x = 0; x < 4 * n; x++) {
        s = s * 6364136223846793005ULL + 1442695040888963407ULL;
        double r = (double)(s >> 11) / 9007199254740992.0 - 0.5;
        if (x < n) u[x] = r; else v[x - n] = r;
    }
    double lam = 0.0;
    for (int it = 0; it < iters; it++) {
        double nrm = 0.0;
        for (long x = 0; x < n; x++) nrm += u[x] * u[x];
        for (long x = 0; x < 3 * n; x++) nrm += v[x] * v[x];
        nrm = sqrt(nrm);
        for (long x = 0; x < n; x++) u[x] /= nrm;
        for (long x = 0; x < 3 * n; x++) v[x] /= nrm;
        or_apply_K(nx, ny, nz, u, v, kp, kq);
        or_apply_KT(nx, ny, nz, kp, kq, u, v);
        double dot = 0.0;
        for (long x = 0; x < n; x++) dot += u[x] * u[x];
        for (long x = 0; x < 3 * n; x++) dot += v[x] * v[x];
        lam = sqrt(dot);
    }
    free(u);
    free(v);
    free(kp);
    free(kq);
    return lam;
}
