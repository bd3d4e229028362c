/*
 * morph.h -- C interface of the MI355X (gfx950) binary morphology library.
 *
 * Operations: erosion, dilation, opening and closing of binary images by
 * rectangular structuring elements, on packed 1-bit bitmaps and on
 * run-length images, plus conversion between the two (Breuel, "Efficient
 * Binary and Run Length Morphology and its Application to Document Image
 * Processing": sections "Run Length Image Coding", "Within-Line
 * Morphological Operations", "Between Line Boolean Operations", "Efficient
 * Binary Decompositions", "2D Morphological Operators for Rectangular
 * Masks", "Conversion Between Image Formats").
 *
 * ----------------------------------------------------------------------------
 * Conventions shared by every entry point
 *
 *  Pixels.  An image has `width` x `height` pixels; row 0 is the first row in
 *  memory; 1 = black = foreground ("in a run").
 *
 *  Structuring element.  morph_se_t {w, h, cx, cy} is the rectangle
 *      B = { (dx,dy) : -cx <= dx <= w-1-cx,  -cy <= dy <= h-1-cy }
 *  with w, h >= 1, 0 <= cx < w, 0 <= cy < h.  The usual centred origin is
 *  (w/2, h/2) rounded down.
 *
 *  Borders.  Erosion treats pixels outside the image as 1, dilation as 0:
 *      erode (x,y) = AND of A over [x-cx, x+w-1-cx] x [y-cy, y+h-1-cy]
 *      dilate(x,y) = OR  of A over [x-(w-1-cx), x+cx] x [y-(h-1-cy), y+cy]
 *  (dilation uses the reflected window: it is the union of B placed at every
 *  black pixel).  open = dilate(erode(A)), close = erode(dilate(A)) with the
 *  same B; each step applies its own outside value to an intermediate that
 *  exists on the image only.
 *
 *  Packed bitmaps (morph_bitmap_t).  Rows of uint64 words; pixel x of row y
 *  is bit (x & 63) of words[y*stride_words + (x >> 6)] (least significant bit
 *  first).  stride_words >= ceil(width/64).  Pad bits (x >= width) and pad
 *  words are ignored on input; on output every bit of word columns
 *  0 .. ceil(width/64)-1 is written, pad bits as 0; words past that in a row
 *  are not touched.  `npages` equal-size pages may be stacked: page p
 *  starts at words + p*height*stride_words and every page is processed on
 *  its own (its own borders).
 *
 *  Run-length images (morph_rle_t).  Row r (r = 0 .. npages*height-1, pages
 *  stacked) holds the runs row_ptr[r] .. row_ptr[r+1]-1; run k is the
 *  half-open interval [runs[2k], runs[2k+1]) of black pixels.  Runs of a row
 *  are ascending, non-empty and separated by at least one white pixel
 *  (end_k < start_{k+1}), which makes the form unique.  Inputs must be in
 *  this form; outputs always are.  `capacity` is the number of runs the
 *  runs array can hold (2*capacity int32).  An output's true run count is
 *  always written to row_ptr[npages*height]; if it exceeds capacity the
 *  runs past capacity are not written and the result is incomplete (check
 *  after the stream has finished; morph_rle_max_runs() is always enough).
 *
 *  Memory.  Every pointer inside the structs, and every workspace, is
 *  device memory owned by the caller.  The structs themselves are read on
 *  the host during the call and may be freed once it returns.  No entry
 *  point allocates device memory, except morph_batch_plan_create (which owns
 *  what it allocates until morph_batch_plan_destroy) and the debugging check
 *  morph_rle_validate.  dst must not overlap
 *  src (MORPH_E_ALIAS).
 *
 *  Streams and errors.  Work is queued on `stream` and runs asynchronously;
 *  a return of MORPH_OK means the work was queued.  Argument errors are
 *  detected on the host before anything is queued and return a negative
 *  code; launch failures return MORPH_E_HIP (morph_last_hip_error() gives the
 *  HIP message of the calling thread's last failure).
 * ----------------------------------------------------------------------------
 */
#ifndef MORPH_H
#define MORPH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t *morph_stream_t;   /* a hipStream_t; NULL = default stream */

enum {
    MORPH_OK = 0,
    MORPH_E_INVAL = -1,          /* null or misaligned pointer, non-positive size, bad element, bad stride */
    MORPH_E_SHAPE = -2,          /* dst and src sizes differ */
    MORPH_E_ALIAS = -3,          /* dst memory overlaps src memory */
    MORPH_E_WORKSPACE = -4,      /* workspace smaller than morph_workspace_bytes() */
    MORPH_E_NONCANONICAL = -5,   /* morph_rle_validate: runs not in the canonical form */
    MORPH_E_CAPACITY = -6,       /* run capacity below what the call can guarantee */
    MORPH_E_HIP = -7,            /* a HIP call failed */
    MORPH_E_UNSUPPORTED = -8     /* outside what the library implements */
};

enum { MORPH_ERODE = 0, MORPH_DILATE = 1, MORPH_OPEN = 2, MORPH_CLOSE = 3 };
enum { MORPH_PACKED = 0, MORPH_RLE = 1 };

typedef struct {
    uint64_t *words;
    int32_t width, height, stride_words;
    int32_t npages;                      /* >= 1 */
} morph_bitmap_t;

typedef struct {
    int32_t width, height;
    int32_t npages;                      /* >= 1 */
    int32_t *row_ptr;                    /* npages*height + 1 entries */
    int32_t *runs;                       /* 2*capacity entries, 8-byte aligned */
    int64_t capacity;
} morph_rle_t;

typedef struct { int32_t w, h, cx, cy; } morph_se_t;

/* ---- library ------------------------------------------------------------ */

/* Version string and a description of the device the library runs on. */
const char *morph_version(void);
/* Message for an error code. */
const char *morph_strerror(int code);
/* Message of the calling thread's last HIP failure ("" if none). */
const char *morph_last_hip_error(void);
/* Copies bytes from src to dst on stream, asynchronously (device memory or
 * pinned host memory on either side), for callers that keep their page
 * buffers in pools, such as a serving loop, and so need none of a framework
 * copy's bookkeeping.  The buffers must stay allocated until the stream has
 * passed the copy.  MORPH_E_INVAL for null pointers with bytes > 0;
 * MORPH_E_HIP if the copy cannot be queued. */
int morph_copy_async(void *dst, const void *src, size_t bytes, morph_stream_t stream);

/* ---- packed bitmaps ----------------------------------------------------- */
/*
 * Rectangle erosion / dilation / opening / closing of packed bitmaps
 * (sections "Efficient Binary Decompositions" and "2D Morphological
 * Operators for Rectangular Masks": separable row and column passes, each a
 * logarithmic decomposition into shifted word-wise AND (erosion) or OR
 * (dilation)).  dst and src must have equal width, height and npages;
 * strides may differ.  ws/ws_bytes: device workspace of at least
 * morph_workspace_bytes(op, MORPH_PACKED, ...) bytes (0 for most elements;
 * ws may then be NULL).  One image of workspace is needed when the
 * operation runs as two launches: an element reaching more than 64 pixels
 * sideways or 128 rows down (split by the composition law), or an opening
 * or closing whose two stages bring more halo rows than 0.6 of the output
 * rows a fused tile holds (51 x 51 on 2550-pixel rows, for instance).  Whether that
 * happens depends on the element and the width only, so the size queried
 * for a stack's total rows covers every page height.
 */
int morph_erode_rect_packed(const morph_bitmap_t *dst, const morph_bitmap_t *src, morph_se_t se,
                            void *ws, size_t ws_bytes, morph_stream_t stream);
int morph_dilate_rect_packed(const morph_bitmap_t *dst, const morph_bitmap_t *src, morph_se_t se,
                             void *ws, size_t ws_bytes, morph_stream_t stream);
int morph_open_rect_packed(const morph_bitmap_t *dst, const morph_bitmap_t *src, morph_se_t se,
                           void *ws, size_t ws_bytes, morph_stream_t stream);
int morph_close_rect_packed(const morph_bitmap_t *dst, const morph_bitmap_t *src, morph_se_t se,
                            void *ws, size_t ws_bytes, morph_stream_t stream);

/*
 * Black pixels of every page: counts[p] (device int64, npages entries,
 * 8-byte aligned) = the number of 1 pixels of page p, pad bits excluded.
 * The input of the choice between the packed and the run-length path by
 * page density (section "Experiments", subsection "2D Rectangular Masks":
 * the representation is picked at run time, conversion costs included).
 * counts must not overlap the image (MORPH_E_ALIAS).
 */
int morph_popcount_pages(const morph_bitmap_t *src, int64_t *counts, morph_stream_t stream);

/* ---- run-length images -------------------------------------------------- */
/*
 * The same four operations on run-length images (section "2D Morphological
 * Operators for Rectangular Masks", third strategy: within-line operations
 * first -- runs shrink, grow and merge, section "Within-Line Morphological
 * Operations" -- then between-line operations, the intersection (erosion)
 * or union (dilation) of the run lists of h consecutive rows, computed by
 * logarithmic decomposition into pairwise merges, sections "Between Line
 * Boolean Operations" and "Efficient Binary Decompositions").
 * Any dst->capacity is accepted: the result's true run count is written to
 * dst->row_ptr[npages*height] and runs past capacity are not written (the
 * caller compares after the stream has passed the call and retries with a
 * larger array; morph_rle_max_runs() never overflows).  The result must have
 * fewer than 2^31 runs.  ws: at least morph_rle_workspace_bytes(op, width,
 * height, npages, se) bytes.
 *
 * Two forms, picked by the workspace given.  The slot form (the fast one)
 * keeps every intermediate row in a workspace slot of ceil(width/2) runs:
 * morph_rle_workspace_bytes() gives its size, about 20 KB per image row at
 * letter width.  It needs the worst case, npages*height*ceil(width/2)
 * runs, and the npages*(height+h-1) extended rows (twice that for elements
 * of 9 or more rows and 2 or more columns) below 2^31.  The band form keeps
 * one band of rows per workgroup with every intermediate row in LDS: a
 * count launch, a scan of the counts into row_ptr, an emit launch; its
 * workspace, morph_rle_workspace_bytes_compact(), is about 12 bytes per row
 * plus a fixed scratch for rows too dense for LDS.  It takes images
 * narrower than 65536 pixels whose element needs at most 383 rows of halo
 * (h - 1, twice that for opening and closing), any number of pages, and
 * runs several times slower.  A workspace of at least the slot size runs
 * the slot form; a smaller one of at least the compact size, 256-byte
 * aligned, the band form (also when the image is too large for the slot
 * form, where morph_rle_workspace_bytes() returns the compact size).
 * Neither possible: MORPH_E_UNSUPPORTED.
 */
int morph_erode_rect_rle(const morph_rle_t *dst, const morph_rle_t *src, morph_se_t se,
                         void *ws, size_t ws_bytes, morph_stream_t stream);
int morph_dilate_rect_rle(const morph_rle_t *dst, const morph_rle_t *src, morph_se_t se,
                          void *ws, size_t ws_bytes, morph_stream_t stream);
int morph_open_rect_rle(const morph_rle_t *dst, const morph_rle_t *src, morph_se_t se,
                        void *ws, size_t ws_bytes, morph_stream_t stream);
int morph_close_rect_rle(const morph_rle_t *dst, const morph_rle_t *src, morph_se_t se,
                         void *ws, size_t ws_bytes, morph_stream_t stream);

/* ---- conversion (section "Conversion Between Image Formats") ------------ */
/*
 * Packed bitmap -> run-length image: the maximal runs of every row.  The run
 * count is written to dst->row_ptr[npages*height] even when it exceeds
 * dst->capacity (then runs past capacity are dropped).  ws: at least
 * morph_pack_to_rle_workspace_bytes(width, height*npages) bytes.
 */
int morph_pack_to_rle(const morph_rle_t *dst, const morph_bitmap_t *src,
                      void *ws, size_t ws_bytes, morph_stream_t stream);
/*
 * Allocation-free morph_pack_to_rle, for callers that cannot allocate device
 * memory or pass a workspace: code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc.  Same arguments, result and run
 * count contract as morph_pack_to_rle, without ws: its scratch (the row
 * counts and the scan's partial sums) is a fixed device array of 16 MiB
 * that the library keeps on every GPU it runs on until the process ends.
 * At most MORPH_NOALLOC_MAX_ROWS rows (npages*height) per call; more
 * returns MORPH_E_UNSUPPORTED before anything is queued.  Every call on one
 * GPU uses that GPU's one array: calls that overlap on a GPU (other
 * streams, other threads) race, so the caller serialises them.  No HIP
 * allocation, free or event creation happens in the call (its launches are
 * not traced).
 */
#define MORPH_NOALLOC_MAX_ROWS 4000000
int morph_pack_to_rle_noalloc(const morph_rle_t *dst, const morph_bitmap_t *src, morph_stream_t stream);
/* Run-length image -> packed bitmap (pad bits 0).  src must be canonical;
 * offsets in row_ptr are clamped to src->capacity.  MORPH_E_UNSUPPORTED when
 * rows * words per row reaches 2^32. */
int morph_rle_to_pack(const morph_bitmap_t *dst, const morph_rle_t *src, morph_stream_t stream);

/* ---- transposition (section "Efficient Transpose") ---------------------- */
/*
 * Transpose of every page: dst row x holds column x of src.  dst->width must
 * equal src->height, dst->height src->width, and npages must agree
 * (MORPH_E_SHAPE otherwise).  Packed: one read of src and one write of dst,
 * pad bits of dst written 0.
 */
int morph_transpose_packed(const morph_bitmap_t *dst, const morph_bitmap_t *src, morph_stream_t stream);
/*
 * Run-length transpose: dst row x holds the runs of column x of src (the
 * runs are decoded into a bitmap, rows of up to 128 words in their own
 * orientation and then transposed 64 x 64 pixels at a time, wider rows
 * straight into the transposed bitmap, which is then re-encoded).  dst->capacity must be at least
 * morph_rle_max_runs(src->height, src->width * npages) (MORPH_E_CAPACITY);
 * ws: 256-byte aligned, at least morph_transpose_rle_workspace_bytes(src
 * width, src height, npages) bytes.
 */
int morph_transpose_rle(const morph_rle_t *dst, const morph_rle_t *src, void *ws, size_t ws_bytes,
                        morph_stream_t stream);
size_t morph_transpose_rle_workspace_bytes(int32_t width, int32_t height, int32_t npages);
/*
 * The rectangle operations on run-length images by within-line operations
 * and transposition (section "2D Morphological Operators for Rectangular
 * Masks", second strategy; the erode2d composition of section "Run Length
 * Image Coding"): the within-line operation along the rows, transpose, the
 * within-line operation along the former columns, transpose back.  Same
 * result as morph_<op>_rect_rle.  op: MORPH_ERODE .. MORPH_CLOSE.
 * dst->capacity as for morph_<op>_rect_rle; ws: 256-byte aligned, at least
 * morph_rlet_workspace_bytes(op, width, height, npages, se) bytes (it holds
 * a run buffer of the worst-case size of the transposed image, about
 * 4 bytes per pixel).  MORPH_E_UNSUPPORTED when that worst case reaches
 * 2^31 runs.
 */
int morph_rect_rlet(int op, const morph_rle_t *dst, const morph_rle_t *src, morph_se_t se, void *ws,
                    size_t ws_bytes, morph_stream_t stream);
size_t morph_rlet_workspace_bytes(int op, int32_t width, int32_t height, int32_t npages, morph_se_t se);

/* ---- components and statistics (sections "Connected Component Extraction
 *      and Statistics", "Other Operations") ----------------------------------- */
/*
 * Connected components of the runs of every page.  Two runs of neighbouring
 * rows touch when their pixel intervals overlap (connectivity 4) or overlap
 * after widening by one pixel (connectivity 8).  labels[i] receives the
 * component number of run i (runs counted over all pages, as in row_ptr),
 * numbered 0, 1, ... within each page in the raster order of each
 * component's first run.  comp_ptr (npages + 1 int32, device) receives the
 * index of each page's first component in a numbering over all pages;
 * comp_ptr[npages] is the total.  labels must hold max_runs int32; runs with
 * index >= max_runs are not labelled and comp_ptr[npages] is set to -1 (check
 * after the stream has passed the call; passing src->capacity is always
 * enough).  ws: 256-byte aligned, morph_rle_label_workspace_bytes(height *
 * npages, max_runs) bytes.  The union-find links are made with atomics, but
 * the labels do not depend on their order.
 */
int morph_rle_label(const morph_rle_t *src, int32_t connectivity, int32_t *labels, int64_t max_runs,
                    int32_t *comp_ptr, void *ws, size_t ws_bytes, morph_stream_t stream);
size_t morph_rle_label_workspace_bytes(int32_t rows, int64_t max_runs);

/* Statistics of one component: bounding box [x0, x1) x [y0, y1) in page
 * coordinates, pixel count and the sums of the pixels' x and y (centroid =
 * sum / area). */
typedef struct {
    int32_t x0, y0, x1, y1;
    int64_t area, sum_x, sum_y;
} morph_component_t;
/* Statistics of the components morph_rle_label found (labels, comp_ptr and
 * max_runs as given to it): stats[c] for component c of the numbering over
 * all pages, c < max_components (components past that are skipped). */
int morph_rle_component_stats(const morph_rle_t *src, const int32_t *labels, int64_t max_runs,
                              const int32_t *comp_ptr, morph_component_t *stats, int64_t max_components,
                              morph_stream_t stream);
/* Run-length histograms per page: black[p * (width + 1) + n] = black runs of
 * length n on page p, white[...] = white runs of length n lying between two
 * black runs of the same row.  Each array: npages * (width + 1) int32,
 * overwritten.  Vertical histograms: transpose first (morph_transpose_rle). */
int morph_rle_run_histograms(const morph_rle_t *src, int32_t *black, int32_t *white, morph_stream_t stream);
/* out[0] = the smallest n at which the running count of the summed
 * histograms hist[p * nbins + n] (p < nrows) reaches num/den of their total
 * (0 for empty histograms); 0 < num <= den <= 2^20; the total must stay
 * below 2^31.  ws: 256-byte aligned, morph_histogram_percentile_workspace_bytes(nbins)
 * bytes (the summed histogram). */
int morph_histogram_percentile(const int32_t *hist, int32_t nrows, int32_t nbins, int32_t num, int32_t den,
                               int32_t *out, void *ws, size_t ws_bytes, morph_stream_t stream);
size_t morph_histogram_percentile_workspace_bytes(int32_t nbins);

/* ---- arbitrary masks (section "Morphology with Arbitrary Masks") -------- */
/*
 * A mask is an h x w array of bytes in host memory (row-major, nonzero =
 * pixel of the mask) with its origin (cx, cy) inside the frame:
 *     erode (x,y) = AND of A(x + i - cx, y + j - cy) over the mask pixels (i, j)
 *     dilate(x,y) = OR  of A(x - i + cx, y - j + cy) over the mask pixels
 * with outside pixels 1 for erosion and 0 for dilation, as for rectangles
 * (a full mask gives the rectangle operations); open and close compose them.
 * An empty mask erodes to all 1s and dilates to all 0s.  The mask is read
 * during the call only.  At most 256 horizontal runs, w and h below 32768
 * (MORPH_E_UNSUPPORTED otherwise, also when a packed tile with the mask's
 * halo does not fit in LDS).
 */
typedef struct {
    const uint8_t *bits;
    int32_t w, h, cx, cy;
} morph_mask_t;
/* Packed: the erosion is one launch that builds the horizontal erosions by
 * 1, 2, 4, ... pixels of a tile in LDS and takes each mask run from the
 * largest one not longer than it, at the run's two ends.  ws: for open and
 * close one intermediate image, morph_mask_workspace_bytes(op, MORPH_PACKED,
 * ...) bytes (256-byte aligned). */
int morph_mask_packed(int op, const morph_bitmap_t *dst, const morph_bitmap_t *src, const morph_mask_t *mask,
                      void *ws, size_t ws_bytes, morph_stream_t stream);
/* Run-length: one pass per mask run, intersecting the accumulated rows with
 * the source rows dy below, eroded along the line by the run.  dst->capacity
 * as for the rectangle operations; ws: morph_mask_workspace_bytes(op,
 * MORPH_RLE, ...) bytes (256-byte aligned). */
int morph_mask_rle(int op, const morph_rle_t *dst, const morph_rle_t *src, const morph_mask_t *mask, void *ws,
                   size_t ws_bytes, morph_stream_t stream);
size_t morph_mask_workspace_bytes(int op, int repr, int32_t width, int32_t height, int32_t npages,
                                  const morph_mask_t *mask);

/* ---- line shifts (section "Scaling, Skewing, and Rotation") ------------- */
/*
 * Every line moves right by its own shift: dst(x, y) = src(x - shifts[r], y)
 * where that lies inside the source line, fill (0 or 1) elsewhere; r counts
 * the rows of all stacked pages.  shifts: device int32, height * npages
 * entries (values are clamped to +-2^30).  dst and src must agree in height
 * and npages; their widths may differ (a skew that keeps every pixel needs a
 * wider destination).  Skews with any slope, skews across the lines (by
 * transposing), rotation by three skews and line operations at an angle
 * are sequences of these calls.
 */
int morph_shift_rows_packed(const morph_bitmap_t *dst, const morph_bitmap_t *src, const int32_t *shifts,
                            int32_t fill, morph_stream_t stream);
/* Run-length form; dst->capacity >= morph_rle_max_runs(dst width, rows);
 * ws: morph_shift_rows_rle_workspace_bytes(height * npages) bytes, 256-byte
 * aligned. */
int morph_shift_rows_rle(const morph_rle_t *dst, const morph_rle_t *src, const int32_t *shifts, int32_t fill,
                         void *ws, size_t ws_bytes, morph_stream_t stream);
size_t morph_shift_rows_rle_workspace_bytes(int32_t rows);

/* ---- skews, rotation, lines at a slope (sections "Scaling, Skewing, and
 *      Rotation", "Morphology with Lines at Arbitrary Orientations") -------- */
/*
 * Compositions of the calls above; the integer shift of every line is
 * computed on the device from the arguments, and the intermediate images
 * live in the workspace (256-byte aligned, at least the bytes the matching
 * *_workspace_bytes function returns; 0 from it means the arguments are
 * invalid or too large).  Run-length destinations need capacity >=
 * morph_rle_max_runs(dst width, dst height * npages).  repr is MORPH_PACKED
 * or MORPH_RLE.
 *
 * Lossless skew.  axis 0 (along the lines): line y of each page moves right
 * by floor(num (y - origin) / den) less the smallest such shift, into a
 * destination wider by morph_skew_spread(height, num, den, origin) pixels
 * (same height).  axis 1 (across the lines): column x moves down by
 * floor(num (x - origin) / den) less the smallest, into a destination taller
 * by morph_skew_spread(width, num, den, origin) (same width); it runs as
 * transpose, skew along the lines, transpose.  Pixels that no source pixel
 * lands on get fill (0 or 1).  den > 0.
 */
int64_t morph_skew_spread(int32_t lines, int32_t num, int32_t den, int32_t origin);
size_t morph_skew_workspace_bytes(int repr, int axis, int32_t width, int32_t height, int32_t npages, int32_t num,
                                  int32_t den, int32_t origin);
int morph_skew_packed(int axis, const morph_bitmap_t *dst, const morph_bitmap_t *src, int32_t num, int32_t den,
                      int32_t origin, int32_t fill, void *ws, size_t ws_bytes, morph_stream_t stream);
int morph_skew_rle(int axis, const morph_rle_t *dst, const morph_rle_t *src, int32_t num, int32_t den,
                   int32_t origin, int32_t fill, void *ws, size_t ws_bytes, morph_stream_t stream);
/*
 * Rotation by `angle` radians (|angle| <= pi/2, else MORPH_E_UNSUPPORTED) as
 * three lossless skews about the frame centre: along the lines by
 * -tan(angle/2), across them by sin(angle), along them by -tan(angle/2),
 * each slope the nearest rational over 2^16 (morph_rotation_rationals with
 * den = 65536 gives the numerators).  Every pixel is kept: the destination
 * is morph_rotate_dims() large; new pixels are 0.
 */
int morph_rotation_rationals(double angle, int32_t den, int32_t *tan_num, int32_t *sin_num);
int morph_rotate_dims(int32_t width, int32_t height, double angle, int32_t *out_width, int32_t *out_height);
size_t morph_rotate_workspace_bytes(int repr, int32_t width, int32_t height, int32_t npages, double angle);
int morph_rotate_packed(const morph_bitmap_t *dst, const morph_bitmap_t *src, double angle, void *ws,
                        size_t ws_bytes, morph_stream_t stream);
int morph_rotate_rle(const morph_rle_t *dst, const morph_rle_t *src, double angle, void *ws, size_t ws_bytes,
                     morph_stream_t stream);
/*
 * Erosion (op MORPH_ERODE) or dilation (MORPH_DILATE) by a centred line of
 * `length` pixels along the slope num/den, |num| <= den (steeper lines:
 * transpose first): the columns are skewed so that the line lies along the
 * rows (column x by -floor(num x / den); pixels brought in from outside
 * take the border value, 1 for erosion and 0 for dilation), the rows get
 * the length x 1 operation, and the inverse skew returns the original
 * frame.  dst has src's size.
 */
size_t morph_line_op_workspace_bytes(int repr, int op, int32_t width, int32_t height, int32_t npages,
                                     int32_t length, int32_t num, int32_t den);
int morph_line_op_packed(int op, const morph_bitmap_t *dst, const morph_bitmap_t *src, int32_t length, int32_t num,
                         int32_t den, void *ws, size_t ws_bytes, morph_stream_t stream);
int morph_line_op_rle(int op, const morph_rle_t *dst, const morph_rle_t *src, int32_t length, int32_t num,
                      int32_t den, void *ws, size_t ws_bytes, morph_stream_t stream);

/*
 * Layout analysis on runs (sections "Connected Component Extraction and
 * Statistics" and "Experiments", the layout use): spacing[0] (host) = the
 * percentile num/den (0 < num <= den <= 2^20) of the horizontal white runs
 * lying between two black runs of a row, over every page; spacing[1] the
 * same for the vertical ones (found by transposing); every page dilated by
 * the centred (spacing[0] + 1) x (spacing[1] + 1) rectangle into `smeared`
 * (same size as src, capacity as for morph_dilate_rect_rle); the connected
 * components of `smeared` (labels, max_runs, comp_ptr as in
 * morph_rle_label, connectivity 4 or 8) and their statistics stats[c] for
 * c < max_components (as morph_rle_component_stats).  Synchronous: the call
 * waits for the stream once, after the spacings, because they set the
 * dilation's element; the rest is queued.  A vertical spacing of 383 or
 * more (a smear too tall for the band form of the dilation) returns
 * MORPH_E_UNSUPPORTED after that wait.  ws: 256-byte aligned,
 * morph_layout_rle_workspace_bytes(width, height, npages, max_runs) bytes.
 */
size_t morph_layout_rle_workspace_bytes(int32_t width, int32_t height, int32_t npages, int64_t max_runs);
int morph_layout_rle(const morph_rle_t *src, int32_t num, int32_t den, int32_t connectivity,
                     const morph_rle_t *smeared, int32_t *labels, int64_t max_runs, int32_t *comp_ptr,
                     morph_component_t *stats, int64_t max_components, int32_t *spacing, void *ws,
                     size_t ws_bytes, morph_stream_t stream);

/* ---- sizes and checks --------------------------------------------------- */
/* Workspace bytes an operation on one page needs (op: MORPH_ERODE ..
 * MORPH_CLOSE; repr: MORPH_PACKED or MORPH_RLE).  For a packed stack pass
 * height*npages; for a run-length stack use morph_rle_workspace_bytes. */
size_t morph_workspace_bytes(int op, int repr, int32_t width, int32_t height, morph_se_t se);
/* Workspace bytes of a run-length operation on npages stacked pages: the
 * slot form's, or the band form's where the slot form cannot take the
 * image.  _compact: the band form's (0 where it does not apply). */
size_t morph_rle_workspace_bytes(int op, int32_t width, int32_t height, int32_t npages, morph_se_t se);
size_t morph_rle_workspace_bytes_compact(int op, int32_t width, int32_t height, int32_t npages, morph_se_t se);
/* Workspace bytes morph_pack_to_rle needs (height counts all stacked pages). */
size_t morph_pack_to_rle_workspace_bytes(int32_t width, int32_t height);
/* Most runs an image of this size can have: height * ceil(width/2). */
int64_t morph_rle_max_runs(int32_t width, int32_t height);
/* Synchronous check (waits for `stream`) that r is canonical, for debugging:
 * MORPH_OK or MORPH_E_NONCANONICAL.  It allocates (and frees) a 4-byte
 * device flag, the one exception to the no-allocation rule besides batch
 * plans. */
int morph_rle_validate(const morph_rle_t *r, morph_stream_t stream);

/* ---- batches of uneven pages (one persistent launch) -------------------- */
/*
 * A batch plan runs many packed pages of different sizes, each with its own
 * operation and element, as one persistent kernel launch (captured in a
 * HIP graph on first run and replayed afterwards).  Tiles of every page go
 * into one work queue; the tile shape per page comes from `tile_rows` /
 * `strip_words` of its descriptor (0 = library default).
 */
typedef struct {
    morph_bitmap_t dst, src;             /* npages must be 1 */
    int32_t op;                          /* MORPH_ERODE .. MORPH_CLOSE */
    morph_se_t se;
    int32_t tile_rows, strip_words;      /* 0 = default */
} morph_page_desc_t;

typedef struct morph_batch_plan morph_batch_plan_t;

/* Builds the tile queue for n pages (descs in host memory) and uploads it.
 * Fails with MORPH_E_UNSUPPORTED for an element the single-launch kernel
 * cannot take (w > 129 or a side of the origin more than 64 pixels wide,
 * or too tall for a tile); run such pages with the per-page calls. */
int morph_batch_plan_create(morph_batch_plan_t **plan, const morph_page_desc_t *descs, int32_t n,
                            morph_stream_t stream);
/* Runs the whole batch: one launch (graph replay when use_graph != 0). */
int morph_batch_run(morph_batch_plan_t *plan, int32_t use_graph, morph_stream_t stream);
/* Number of tiles in the plan. */
int64_t morph_batch_tiles(const morph_batch_plan_t *plan);
void morph_batch_plan_destroy(morph_batch_plan_t *plan);

/*
 * The same persistent launch without a plan, for batches that change from
 * call to call (a serving loop): the tile tables are built on the host and
 * copied into the caller's device workspace `ws` (256-byte aligned, at least
 * morph_batch_workspace_bytes(descs, n) bytes) before the launch, all on
 * `stream`.  host_staging, if not NULL, is caller-owned pinned host memory of
 * the same size that the copy reads from asynchronously: it must stay
 * untouched until the stream has passed this call.  With host_staging NULL
 * the tables are copied from library memory and the call waits for the copy.
 * Returns -1 from morph_batch_workspace_bytes for descriptors the batch
 * kernel cannot take (see morph_batch_plan_create).
 */
int64_t morph_batch_workspace_bytes(const morph_page_desc_t *descs, int32_t n);
int morph_batch_launch(const morph_page_desc_t *descs, int32_t n, void *ws, size_t ws_bytes,
                       void *host_staging, size_t staging_bytes, morph_stream_t stream);

/* ---- tracing (benchmarks and profiling) --------------------------------- */
/*
 * While tracing is on, the library records a pair of HIP events around every
 * launch of the kernels below, on the stream of the call, and the run-length
 * kernels add the runs they read and write to counters in the device buffer
 * given to morph_trace_begin.  morph_trace_end waits for the stream and
 * returns, per kernel, the number of launches, the summed event-measured
 * duration and the algorithmic bytes: what the operation has to move, i.e.
 * one read of its input and one write of its output (packed: 8 bytes per
 * word; runs: 8 bytes per run plus 4 per row count), not what the kernel
 * happens to re-read.  Tracing state is process-wide: trace one thread at a
 * time.
 */
enum {
    MORPH_K_RECT = 0,          /* fused packed rectangle kernel (per-op launches) */
    MORPH_K_RECT_BATCH = 1,    /* persistent batched packed kernel */
    MORPH_K_PACK_TO_RLE = 2,   /* bitmap -> runs (count and emit launches) */
    MORPH_K_RLE_TO_PACK = 3,   /* runs -> bitmap */
    MORPH_K_ROW_ERODE = 4,     /* within-line pass on runs (elements one row tall) */
    MORPH_K_COL_AND = 5,       /* between-line doubling step on runs; the first step of a
                                  chain also applies the within-line pass to the rows it reads */
    MORPH_K_PACK_ROWS = 6,     /* final packing of run rows into CSR */
    MORPH_K_TRANSPOSE = 7,     /* packed bitmap -> its transpose */
    MORPH_K_DECODE_T = 8,      /* runs -> transposed packed bitmap, with a within-line
                                  operation applied to the runs as they are read */
    MORPH_K_COMPONENTS = 9,    /* connected-component labelling of runs (all its launches) */
    MORPH_K_COMPONENT_STATS = 10, /* per-component box, area and coordinate sums */
    MORPH_K_HISTOGRAM = 11,    /* run-length histograms */
    MORPH_K_MASK = 12,         /* packed erosion by an arbitrary mask */
    MORPH_K_MASK_RLE = 13,     /* intersection with one eroded, shifted mask run on runs */
    MORPH_K_SHIFT = 14,        /* packed line shifts */
    MORPH_K_SHIFT_RLE = 15,    /* line shifts on runs (count and emit launches) */
    MORPH_K_COL_SCAN = 16,     /* between-line block prefix scans on runs (tall elements) */
    MORPH_K_RLE_BAND = 17,     /* run-length rectangle operation, one band per workgroup in LDS:
                                  the launch that writes the runs */
    MORPH_K_RLE_BAND_COUNT = 18, /* the same, the launch that counts each output row's runs */
    MORPH_K_TRANSPOSE_TO_RLE = 19, /* bitmap -> runs of its transpose: the transpose with the run
                                     counts of its rows, the scan, the emit launch */
    MORPH_K_COUNT = 20
};
typedef struct {
    int64_t launches;
    double ms;                  /* sum of event-measured launch durations */
    double bytes;               /* algorithmic bytes over all launches */
} morph_kernel_trace_t;
/* Device memory the counters need (128-byte aligned). */
#define MORPH_TRACE_BYTES (MORPH_K_COUNT * 2 * 256 * 128)
/* dev_counters: at least MORPH_TRACE_BYTES of device memory, used until
 * morph_trace_end. */
int morph_trace_begin(void *dev_counters, size_t bytes, morph_stream_t stream);
/* out: MORPH_K_COUNT entries. */
int morph_trace_end(morph_kernel_trace_t *out, morph_stream_t stream);
/* Name of a kernel id. */
const char *morph_kernel_name(int kernel);

#ifdef __cplusplus
}
#endif

#endif /* MORPH_H */
