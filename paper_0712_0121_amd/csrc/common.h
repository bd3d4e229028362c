// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "../../include/morph.h"

namespace morph {

// Workgroups are dealt to the 8 XCDs round robin, and each XCD has its own
// L2.  Kernels whose neighbouring rows share cache lines (a row and the row
// K below it, or the partial lines where one row's runs end and the next
// row's begin) take their rows from this logical index instead of
// blockIdx.x: it gives every XCD one contiguous range of blocks.
__device__ __forceinline__ unsigned xcd_block()
{
    const unsigned n = gridDim.x, b = blockIdx.x;
    const unsigned x = b & 7u, q = n >> 3, rem = n & 7u;
    return x * q + min(x, rem) + (b >> 3);
}

// Value of lane (this lane ^ J) for J = 1, 2, 4, 8 (DPP moves inside the
// 16-lane rows) and 16 (gfx950's v_permlane16_swap: with both operands v it
// returns, for every lane, row 2k of v in its first and row 2k + 1 in its
// second result, k = lane / 32).
template <int J>
__device__ __forceinline__ uint32_t lane_xor(uint32_t v)
{
    static_assert(J == 1 || J == 2 || J == 4 || J == 8 || J == 16, "lane distance");
    if constexpr (J == 1) {
        return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xf, 0xf, false);   // quad_perm 1,0,3,2
    } else if constexpr (J == 2) {
        return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xf, 0xf, false);   // quad_perm 2,3,0,1
    } else if constexpr (J == 4) {
        // row_ror:n reads lane (i - n) mod 16 of the row
        const uint32_t below = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x124, 0xf, 0xf, false);  // i - 4
        const uint32_t above = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x12C, 0xf, 0xf, false);  // i + 4
        return (threadIdx.x & 4) ? below : above;
    } else if constexpr (J == 8) {
        return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x128, 0xf, 0xf, false);  // row_ror:8
    } else {
        const auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);
        return (threadIdx.x & 16) ? r[0] : r[1];
    }
}

// 32-bit bit select: bits of a where k is 1, of b where it is 0 (v_bfi).
__device__ __forceinline__ uint32_t bitsel(uint32_t k, uint32_t a, uint32_t b) { return (a & k) | (b & ~k); }

// One butterfly step: the lane without bit J keeps the bits of m and takes
// its partner's other bits shifted up by J; the lane with bit J keeps the
// bits of ~m and takes its partner's shifted down.  Written branch-free (a
// per-lane all-ones/zero mask and bit selects): as a conditional, both arms
// are taken by half the lanes each and the wave runs both.
template <int J>
__device__ __forceinline__ uint64_t transpose_step(uint64_t x, uint64_t m)
{
    const uint64_t y = ((uint64_t)lane_xor<J>((uint32_t)(x >> 32)) << 32) | lane_xor<J>((uint32_t)x);
    const uint64_t up = 0ull - (uint64_t)((threadIdx.x / J) & 1u);      // all ones on the lane with bit J
    const uint64_t keep = m ^ up;                                       // the bits this lane keeps
    const uint64_t dn = y >> J, upv = y << J;
    const uint64_t ys = ((uint64_t)bitsel((uint32_t)(up >> 32), (uint32_t)(dn >> 32), (uint32_t)(upv >> 32)) << 32) |
                        bitsel((uint32_t)up, (uint32_t)dn, (uint32_t)upv);
    return ((uint64_t)bitsel((uint32_t)(keep >> 32), (uint32_t)(x >> 32), (uint32_t)(ys >> 32)) << 32) |
           bitsel((uint32_t)keep, (uint32_t)x, (uint32_t)ys);
}

// Transposes the 64 x 64 bit matrix a wave holds one row per lane (bit k of
// lane i is element (i, k)): afterwards lane i holds column i.  Six steps;
// step J exchanges the off-diagonal J x J blocks of every 2J x 2J block
// between lanes i and i ^ J.  For J = 32 those blocks are whole 32-bit
// halves: the high half of lanes 0..31 trades places with the low half of
// lanes 32..63, which is one v_permlane32_swap of (low, high).  Every lane
// of the wave must be active.
__device__ __forceinline__ uint64_t wave_transpose64(uint64_t x)
{
    const auto h = __builtin_amdgcn_permlane32_swap((uint32_t)x, (uint32_t)(x >> 32), false, false);
    x = ((uint64_t)h[1] << 32) | h[0];
    x = transpose_step<16>(x, 0x0000ffff0000ffffull);
    x = transpose_step<8>(x, 0x00ff00ff00ff00ffull);
    x = transpose_step<4>(x, 0x0f0f0f0f0f0f0f0full);
    x = transpose_step<2>(x, 0x3333333333333333ull);
    x = transpose_step<1>(x, 0x5555555555555555ull);
    return x;
}

// ------------------------------------------------------------------ packed
// Geometry of the fused band kernel (one workgroup = one tile).
constexpr int kThreads = 512;          // threads per workgroup (large tiles)
constexpr int kLdsWords = 10236;       // ~80 KiB of LDS per workgroup (two per CU, with room for a queue slot)
constexpr int kThreadsSmall = 256;     // threads per workgroup (small tiles: four workgroups per CU)
constexpr int kLdsWordsSmall = 5116;   // ~40 KiB of LDS per small-tile workgroup

constexpr int lds_words_for(int nt) { return nt == kThreadsSmall ? kLdsWordsSmall : kLdsWords; }
constexpr int kChunkMax = 20;          // rows a thread keeps in registers in the column pass
constexpr int kWordsPerItem = 4;       // consecutive words one row-pass item produces
constexpr int kItemsMax = 4;           // row-pass items a thread holds across a barrier
constexpr int kReachMax = 64;          // pixels each side of the origin one pass can reach (row)
constexpr int kStripMax = 64;          // default widest strip (words)

// One erosion pass ("stage") of a rectangle operation.  Every operation is
// run as erosions: dilation_B(A) = not erosion_B^(not A), with B^ the
// reflected element, so outside pixels are always 1 inside the kernel.
struct Stage {
    int w, h, cx, cy;
};

// One page of a rectangle operation as the kernel sees it.
struct RectPage {
    const uint64_t *src;
    uint64_t *dst;
    int W, H, nw;             // pixels, rows, words per row = ceil(W/64)
    int sstride, dstride;     // words
    int nst;                  // 1 or 2 stages fused in the launch
    Stage st[2];
    int in_c, mid_c, out_c;   // complement the input / between stages / the output (0 or 1)
    int TR, SW;               // tile rows, strip words
    int nt;                   // threads per workgroup: kThreads or kThreadsSmall
    int nbands, nstrips;
    uint64_t padmask;         // valid bits of the last word of a row
    long long src_page_words, dst_page_words;  // stacked pages
};

// Tile planning (host) for workgroups of nt threads.  Returns false if no
// tile shape fits.
bool plan_tiles(RectPage &p, int tile_rows, int strip_words, int npages, int nt = kThreads);
bool tile_fits(const RectPage &p);

// Launch one fused pass over npages stacked pages.
hipError_t launch_rect(const RectPage &p, int npages, hipStream_t stream);

// Batched form: a device table of pages and a tile list.
struct TileRef {
    int page, band, strip, pad;
};
hipError_t launch_rect_batch(const RectPage *pages_dev, const TileRef *tiles_dev, int ntiles,
                             int *queue_dev, int nblocks, hipStream_t stream, double alg_bytes);
hipError_t launch_reset_counter(int *queue_dev, hipStream_t stream);
int device_cu_count();

// counts[p] = black pixels of page p (pad bits excluded).
hipError_t popcount_pages(const morph_bitmap_t &src, unsigned long long *counts, hipStream_t stream);

// Transpose of every page of a packed bitmap (dst: width = src height,
// height = src width).
hipError_t packed_transpose(const morph_bitmap_t &dst, const morph_bitmap_t &src, hipStream_t stream);
// The same (untraced), also writing the number of runs that start in each
// piece of every transposed row: counts[piece * rows + row] for the
// transpose_pieces(src height) pieces of a row, consecutive ranges of its
// pixels.
int transpose_pieces(int height);
hipError_t packed_transpose_counted(const morph_bitmap_t &dst, const morph_bitmap_t &src, int *counts,
                                    hipStream_t stream);

// ------------------------------------------------------------ arbitrary masks
// The horizontal runs of a mask as offsets from its origin: run q covers
// the pixels (dx[q] .. dx[q] + len[q] - 1, dy[q]) relative to the origin.
constexpr int kMaskMaxRuns = 256;
struct MaskRunsArg {
    int n;
    short dx[kMaskMaxRuns], dy[kMaskMaxRuns], len[kMaskMaxRuns];
};

// One erosion by a mask of npages stacked packed pages (complementing the
// input and output when in_c / out_c), tiled as TR rows x SW words.
struct MaskPage {
    const uint64_t *src;
    uint64_t *dst;
    int W, H, nw, sstride, dstride;
    long long spw, dpw;
    int in_c, out_c;
    uint64_t padmask;
    int TR, SW, nbands, nstrips;
    int HL, HR, dy0, NR, NW, levels;    // halo words, first row offset, LDS rows and words, doubling levels
};
bool plan_mask(MaskPage &p, const MaskRunsArg &m);
hipError_t launch_mask(const MaskPage &p, const MaskRunsArg &m, int npages, hipStream_t stream);

// ------------------------------------------------------------- run-length
hipError_t rle_from_packed(const morph_rle_t &dst, const morph_bitmap_t &src, void *ws,
                           hipStream_t stream, bool traced = true);
// rle_from_packed with its scratch in the library's fixed device array
// (no allocation); rows = npages * height must be at most
// MORPH_NOALLOC_MAX_ROWS.
hipError_t rle_from_packed_noalloc(const morph_rle_t &dst, const morph_bitmap_t &src, hipStream_t stream);
hipError_t rle_to_packed(const morph_bitmap_t &dst, const morph_rle_t &src, hipStream_t stream);
size_t rle_op_workspace(int op, int32_t W, int32_t rows, int32_t H, morph_se_t se);
// The band form of the rectangle operations on runs (every intermediate in
// LDS): whether it takes (op, width, element), its workspace, the launch.
bool rle_band_applies(int op, int32_t W, morph_se_t se);
size_t rle_band_workspace(int op, int32_t W, long long rows, morph_se_t se);
hipError_t rle_band_op(int op, const morph_rle_t &dst, const morph_rle_t &src, morph_se_t se, void *ws,
                       hipStream_t stream);
bool rle_uses_scan(morph_se_t se);   // between-line pass by block prefix scans
hipError_t rle_rect_op(int op, const morph_rle_t &dst, const morph_rle_t &src, morph_se_t se,
                       void *ws, size_t ws_bytes, hipStream_t stream);
size_t scan_workspace(int64_t n);
hipError_t shift_rows_packed(const morph_bitmap_t &dst, const morph_bitmap_t &src, const int *shifts, int fill,
                             hipStream_t s);
size_t shift_rows_rle_workspace(long long rows);
hipError_t shift_rows_rle(const morph_rle_t &dst, const morph_rle_t &src, const int *shifts, int fill, void *ws,
                          hipStream_t s);
size_t rle_mask_workspace(int W, long long rows);
hipError_t rle_mask_op(int op, const morph_rle_t &dst, const morph_rle_t &src, const MaskRunsArg &m,
                       const MaskRunsArg &reflected, void *ws, hipStream_t s);
// out[0..n] = exclusive scan of in[0..n-1], out[n] = total; tmp holds
// scan_workspace(n) bytes.
hipError_t exclusive_scan(const int *in, int n, int *out, int *tmp, hipStream_t s);

// Connected components of a run-length image (runs with index >= nmax are
// left out; comp_ptr[npages] is then -1), their statistics, and run-length
// histograms.
size_t cc_workspace(long long rows, long long nruns);
hipError_t cc_label(const morph_rle_t &src, int connectivity, int *labels, long long nmax, int *comp_ptr,
                    void *ws, hipStream_t s);
hipError_t cc_stats(const morph_rle_t &src, const int *labels, long long nmax, const int *comp_ptr,
                    morph_component_t *st, long long ncap, hipStream_t s);
hipError_t run_histograms(const morph_rle_t &src, int *black, int *white, hipStream_t s);
size_t percentile_workspace(int nbins);
hipError_t histogram_percentile(const int *hist, int nrows, int nbins, int num, int den, int *out, void *ws,
                                hipStream_t s);

// Within-line operation applied to every run (or, with comp, every gap) of
// a row as it is decoded: erosion shrinks an interval, dilation grows it,
// opening does both.  w, c: element length and origin along the line.
enum { kLineNone = 0, kLineErode = 1, kLineDilate = 2, kLineOpen = 3 };
struct LineOp {
    int mode, w, c, comp;
};
// Runs -> transposed packed bitmap (dst: width = src height, height = src
// width), with op applied along the source rows.
// tmp: a bitmap of src's own size (stride ceil(width/64)), used for rows of
// up to 128 words (decode, then transpose); nullptr keeps the direct decode.
hipError_t rle_decode_transposed(const morph_bitmap_t &dst, const morph_rle_t &src, LineOp op,
                                 hipStream_t stream, uint64_t *tmp = nullptr);
// Runs -> packed bitmap in the runs' own orientation, with op applied along
// the rows (rows of up to 128 words).
hipError_t rle_decode_rows(const morph_bitmap_t &dst, const morph_rle_t &src, LineOp op, hipStream_t stream);
// The runs of the transpose of a packed bitmap (dst: width = src height,
// height = src width, at most 8192): the transpose, with the run counts of
// its rows, into tbuf (a bitmap of the transpose's shape, stride
// ceil(src height / 64)), then the runs from there; ws holds
// transposed_rle_workspace(src width, src height, npages) bytes, 256-aligned.
size_t transposed_rle_workspace(int W, int H, int P);
hipError_t rle_from_packed_transposed(const morph_rle_t &dst, const morph_bitmap_t &src, uint64_t *tbuf, void *ws,
                                      hipStream_t stream);
int rle_validate(const morph_rle_t &r, hipStream_t stream, hipError_t *err);

void set_hip_error(hipError_t e);

// Tracing: events around launches while on; run counters for the
// run-length kernels (device address, or nullptr when tracing is off).
bool trace_on();
void trace_before(int kernel, hipStream_t s);
void trace_after(int kernel, hipStream_t s, double alg_bytes);
unsigned long long *trace_counters();   // [kernel*2] runs read, [kernel*2+1] runs written

}  // namespace morph
