/*
 * CPU oracle for rectangular binary morphology, packing and run-length
 * coding.  TEST INFRASTRUCTURE ONLY: nothing in the product path links,
 * loads or calls this file; only the tests, the smoke check and the CPU
 * baseline leg of the benchmark do.  It shares no code with the HIP path.
 *
 * Everything here is the plain definition, written for a reader to check
 * by eye, not for speed (paper, section "2D Morphological Operators for
 * Rectangular Masks": the brute-force strategy, one shifted AND/OR per
 * mask pixel, is the one meant "for reference and verification").
 *
 * Conventions (the paper leaves them open; this is the reading used
 * throughout):
 *  - image: uint8, H rows of W pixels, row-major, 1 = black = "in a run"
 *    (section "Run Length Image Coding");
 *  - structuring element B(w,h,cx,cy) = { (dx,dy) : -cx <= dx <= w-1-cx,
 *    -cy <= dy <= h-1-cy }, origin (cx,cy) inside the rectangle;
 *  - erosion treats pixels outside the image as 1, dilation as 0;
 *  - dilation is the Minkowski adjoint of erosion: its window is the
 *    erosion window reflected through the origin;
 *  - opening = dilation(erosion(A)), closing = erosion(dilation(A)), both
 *    with the same B; the intermediate is an image on the domain only, so
 *    the second step applies its own outside value;
 *  - packed rows: uint64 words, pixel x is bit (x & 63) of word (x >> 6),
 *    stride >= ceil(W/64) words; pad bits are ignored when unpacking and
 *    written 0 when packing;
 *  - run-length rows: half-open intervals [start,end) of 1s, maximal and
 *    ascending (end_j < start_{j+1}), stored CSR: row_ptr[H+1] and
 *    runs[2*n] = (start,end) pairs.
 */
#include <stdint.h>
#include <stddef.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Number of threads the OpenMP loops below use. */
int oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Sets that number (n >= 1), for timing the oracle on one thread. */
void oracle_set_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

#define PIX(img, W, x, y) ((img)[(size_t)(y) * (size_t)(W) + (size_t)(x)])

/* Erosion by brute force: out(x,y) = 1 iff every pixel of the window
 * [x-cx, x+w-1-cx] x [y-cy, y+h-1-cy] is 1, where pixels outside the
 * image count as 1. */
void oracle_erode(uint8_t *out, const uint8_t *in, int W, int H,
                  int w, int h, int cx, int cy)
{
    #pragma omp parallel for schedule(dynamic, 8)
    for (int y = 0; y < H; y++) {
        for (int x = 0; x < W; x++) {
            int v = 1;
            for (int yy = y - cy; v && yy <= y + h - 1 - cy; yy++) {
                if (yy < 0 || yy >= H) continue;          /* outside: 1 */
                for (int xx = x - cx; xx <= x + w - 1 - cx; xx++) {
                    if (xx < 0 || xx >= W) continue;      /* outside: 1 */
                    if (!PIX(in, W, xx, yy)) { v = 0; break; }
                }
            }
            PIX(out, W, x, y) = (uint8_t)v;
        }
    }
}

/* Dilation by brute force: out(x,y) = 1 iff some pixel of the reflected
 * window [x-(w-1-cx), x+cx] x [y-(h-1-cy), y+cy] is 1, where pixels
 * outside the image count as 0.  Equivalently, out is the union of the
 * translates B + p over all black pixels p. */
void oracle_dilate(uint8_t *out, const uint8_t *in, int W, int H,
                   int w, int h, int cx, int cy)
{
    #pragma omp parallel for schedule(dynamic, 8)
    for (int y = 0; y < H; y++) {
        for (int x = 0; x < W; x++) {
            int v = 0;
            for (int yy = y - (h - 1 - cy); !v && yy <= y + cy; yy++) {
                if (yy < 0 || yy >= H) continue;          /* outside: 0 */
                for (int xx = x - (w - 1 - cx); xx <= x + cx; xx++) {
                    if (xx < 0 || xx >= W) continue;      /* outside: 0 */
                    if (PIX(in, W, xx, yy)) { v = 1; break; }
                }
            }
            PIX(out, W, x, y) = (uint8_t)v;
        }
    }
}

/* Opening and closing: composition of the two definitions above.  tmp is
 * a caller-provided W*H scratch image. */
void oracle_open(uint8_t *out, const uint8_t *in, uint8_t *tmp, int W, int H,
                 int w, int h, int cx, int cy)
{
    oracle_erode(tmp, in, W, H, w, h, cx, cy);
    oracle_dilate(out, tmp, W, H, w, h, cx, cy);
}

void oracle_close(uint8_t *out, const uint8_t *in, uint8_t *tmp, int W, int H,
                  int w, int h, int cx, int cy)
{
    oracle_dilate(tmp, in, W, H, w, h, cx, cy);
    oracle_erode(out, tmp, W, H, w, h, cx, cy);
}

/* Independent evaluator: a summed-area table of black pixels.  S has
 * (H+1)*(W+1) entries, S[y][x] = number of black pixels in [0,x) x [0,y). */
static int64_t sat_box(const int64_t *S, int W, int H,
                       int x0, int x1, int y0, int y1, int64_t *area)
{
    /* count of black pixels and of in-image pixels in the inclusive box
     * [x0,x1] x [y0,y1] clipped to the image */
    if (x0 < 0) x0 = 0;
    if (y0 < 0) y0 = 0;
    if (x1 > W - 1) x1 = W - 1;
    if (y1 > H - 1) y1 = H - 1;
    if (x0 > x1 || y0 > y1) { *area = 0; return 0; }
    *area = (int64_t)(x1 - x0 + 1) * (int64_t)(y1 - y0 + 1);
    const size_t s = (size_t)W + 1;
    return S[(size_t)(y1 + 1) * s + (x1 + 1)] - S[(size_t)y0 * s + (x1 + 1)]
         - S[(size_t)(y1 + 1) * s + x0] + S[(size_t)y0 * s + x0];
}

void oracle_sat_build(int64_t *S, const uint8_t *in, int W, int H)
{
    const size_t s = (size_t)W + 1;
    for (int x = 0; x <= W; x++) S[x] = 0;
    for (int y = 0; y < H; y++) {
        int64_t rowsum = 0;
        S[(size_t)(y + 1) * s] = 0;
        for (int x = 0; x < W; x++) {
            rowsum += PIX(in, W, x, y);
            S[(size_t)(y + 1) * s + (x + 1)] = S[(size_t)y * s + (x + 1)] + rowsum;
        }
    }
}

/* Erosion via the table: 1 iff the clipped window holds no white pixel. */
void oracle_sat_erode(uint8_t *out, const int64_t *S, int W, int H,
                      int w, int h, int cx, int cy)
{
    #pragma omp parallel for schedule(static)
    for (int y = 0; y < H; y++)
        for (int x = 0; x < W; x++) {
            int64_t area;
            int64_t black = sat_box(S, W, H, x - cx, x + w - 1 - cx,
                                    y - cy, y + h - 1 - cy, &area);
            PIX(out, W, x, y) = (uint8_t)(black == area);
        }
}

/* Dilation via the table: 1 iff the clipped reflected window holds a
 * black pixel. */
void oracle_sat_dilate(uint8_t *out, const int64_t *S, int W, int H,
                       int w, int h, int cx, int cy)
{
    #pragma omp parallel for schedule(static)
    for (int y = 0; y < H; y++)
        for (int x = 0; x < W; x++) {
            int64_t area;
            int64_t black = sat_box(S, W, H, x - (w - 1 - cx), x + cx,
                                    y - (h - 1 - cy), y + cy, &area);
            PIX(out, W, x, y) = (uint8_t)(black > 0);
        }
}

/* Packing: pixel x of row y goes to bit (x & 63) of word y*stride + (x>>6);
 * every other bit is 0. */
void oracle_pack(uint64_t *words, const uint8_t *in, int W, int H, int stride)
{
    for (int y = 0; y < H; y++) {
        for (int j = 0; j < stride; j++) words[(size_t)y * stride + j] = 0;
        for (int x = 0; x < W; x++)
            if (PIX(in, W, x, y))
                words[(size_t)y * stride + (x >> 6)] |= (uint64_t)1 << (x & 63);
    }
}

/* Unpacking: the inverse; pad bits (x >= W) are not read. */
void oracle_unpack(uint8_t *out, const uint64_t *words, int W, int H, int stride)
{
    for (int y = 0; y < H; y++)
        for (int x = 0; x < W; x++)
            PIX(out, W, x, y) =
                (uint8_t)((words[(size_t)y * stride + (x >> 6)] >> (x & 63)) & 1);
}

/* Run-length encoding, first pass: number of maximal runs per row, i.e.
 * the number of positions where a 1 follows a 0 or the left border.
 * counts has H entries; returns the total. */
int64_t oracle_rle_count(int32_t *counts, const uint8_t *in, int W, int H)
{
    int64_t total = 0;
    for (int y = 0; y < H; y++) {
        int32_t n = 0;
        for (int x = 0; x < W; x++)
            if (PIX(in, W, x, y) && (x == 0 || !PIX(in, W, x - 1, y))) n++;
        counts[y] = n;
        total += n;
    }
    return total;
}

/* Run-length encoding, second pass: fills row_ptr[H+1] and runs[2*total]
 * with the maximal runs, scanned left to right. */
void oracle_rle_encode(int32_t *row_ptr, int32_t *runs, const uint8_t *in,
                       int W, int H)
{
    int32_t k = 0;
    row_ptr[0] = 0;
    for (int y = 0; y < H; y++) {
        int x = 0;
        while (x < W) {
            if (!PIX(in, W, x, y)) { x++; continue; }
            int s = x;
            while (x < W && PIX(in, W, x, y)) x++;
            runs[2 * k] = s;
            runs[2 * k + 1] = x;      /* half-open end */
            k++;
        }
        row_ptr[y + 1] = k;
    }
}

/* Run-length decoding: every pixel of every run is set, all others are 0. */
void oracle_rle_decode(uint8_t *out, const int32_t *row_ptr, const int32_t *runs,
                       int W, int H)
{
    for (int y = 0; y < H; y++) {
        for (int x = 0; x < W; x++) PIX(out, W, x, y) = 0;
        for (int32_t k = row_ptr[y]; k < row_ptr[y + 1]; k++)
            for (int x = runs[2 * k]; x < runs[2 * k + 1]; x++)
                PIX(out, W, x, y) = 1;
    }
}
