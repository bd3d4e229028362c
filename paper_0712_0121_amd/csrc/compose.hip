// Compositions of the library's operations (section "Scaling, Skewing, and
// Rotation" and section "Morphology with Lines at Arbitrary Orientations"):
// lossless skews along and across the lines, rotation by three skews, and
// erosion or dilation by a line at a slope.  Every step is one of the
// public entry points (line shifts, transposes, rectangle operations); this
// file computes the integer shift of each line on the device and lays the
// intermediate images out in the caller's workspace.
#include "common.h"

#include <algorithm>
#include <cmath>

namespace morph {

namespace {

long long floor_div(long long a, long long b)
{
    long long q = a / b;
    if ((a % b) != 0 && ((a < 0) != (b < 0))) q--;
    return q;
}

__device__ __forceinline__ long long dfloor_div(long long a, long long b)
{
    long long q = a / b;
    if ((a % b) != 0 && ((a < 0) != (b < 0))) q--;
    return q;
}

// shifts[r] for the lines r of all pages, line y = r mod n of its page:
//   skew:      floor(num (y - origin) / den) - vmin
//   line, out: -floor(num y / den) + off
//   line, in:  floor(num y / den) - off
enum { kShiftSkew = 0, kShiftLineOut = 1, kShiftLineIn = 2 };
__global__ void line_shifts_kernel(int *__restrict__ shifts, long long R, int n, int mode, int num, int den,
                                   int origin, long long add)
{
    const long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= R) return;
    const long long y = r % n;
    long long v;
    if (mode == kShiftSkew) v = dfloor_div((long long)num * (y - origin), den) - add;
    else if (mode == kShiftLineOut) v = -dfloor_div((long long)num * y, den) + add;
    else v = dfloor_div((long long)num * y, den) - add;
    shifts[r] = (int)v;
}

hipError_t fill_shifts(int *shifts, long long R, int n, int mode, int num, int den, int origin, long long add,
                       hipStream_t s)
{
    if (R <= 0) return hipSuccess;
    hipLaunchKernelGGL(line_shifts_kernel, dim3((unsigned)((R + 255) / 256)), dim3(256), 0, s, shifts, R, n, mode,
                       num, den, origin, add);
    return hipGetLastError();
}

size_t r256(size_t b) { return (b + 255) & ~(size_t)255; }
size_t bitmap_bytes(int W, long long rows) { return (size_t)((W + 63) / 64) * (size_t)rows * 8; }

// The smallest shift of a skew of n lines and the spread (largest less
// smallest): the shift is monotone in y, so the ends decide.
void skew_range(int n, int num, int den, int origin, long long &vmin, long long &spread)
{
    const long long a = floor_div((long long)num * (0 - origin), den);
    const long long b = floor_div((long long)num * (n - 1 - (long long)origin), den);
    vmin = std::min(a, b);
    spread = std::max(a, b) - vmin;
}

// Run-length images of worst-case capacity carved from the workspace.
size_t rle_bytes(int W, long long rows)
{
    return r256((size_t)(rows + 1) * 4) + r256((size_t)rows * ((W + 1) / 2) * 8);
}

morph_rle_t rle_at(char *p, int W, int H, int P)
{
    const long long rows = (long long)H * P;
    return morph_rle_t{W, H, P, (int32_t *)p, (int32_t *)(p + r256((size_t)(rows + 1) * 4)),
                       rows * ((W + 1) / 2)};
}

bool dims_ok(long long W, long long H, long long P)
{
    return W >= 1 && H >= 1 && P >= 1 && W < (1LL << 30) && H < (1LL << 30) && W * P < (1LL << 31) &&
           H * P < (1LL << 31);
}

// ---------------------------------------------------------------- skews
struct SkewPlan {
    long long vmin, spread;
    size_t shifts, inner, total;   // shift table, the entry point's own workspace
};

SkewPlan skew_rows_plan(int repr, int W, int H, int P, int num, int den, int origin)
{
    SkewPlan k{};
    skew_range(H, num, den, origin, k.vmin, k.spread);
    k.shifts = r256((size_t)H * P * 4);
    k.inner = repr == MORPH_RLE ? r256(morph_shift_rows_rle_workspace_bytes(H * P)) : 0;
    k.total = k.shifts + k.inner;
    return k;
}

int skew_rows_run(int repr, const void *dst, const void *src, int W, int H, int P, int num, int den, int origin,
                  int fill, char *ws, const SkewPlan &k, hipStream_t s)
{
    int *shifts = (int *)ws;
    hipError_t e = fill_shifts(shifts, (long long)H * P, H, kShiftSkew, num, den, origin, k.vmin, s);
    if (e != hipSuccess) { set_hip_error(e); return MORPH_E_HIP; }
    if (repr == MORPH_PACKED)
        return morph_shift_rows_packed((const morph_bitmap_t *)dst, (const morph_bitmap_t *)src, shifts, fill,
                                       (morph_stream_t)s);
    return morph_shift_rows_rle((const morph_rle_t *)dst, (const morph_rle_t *)src, shifts, fill, ws + k.shifts,
                                k.inner, (morph_stream_t)s);
}

// Across the lines: transpose, skew along the lines, transpose back.  The
// workspace holds the two transposed images, then the skew's own
// workspace and the run-length transposes' scratch.
struct ColPlan {
    SkewPlan rows;
    long long spread;
    size_t t1, t2, tr, total;
};

ColPlan skew_cols_plan(int repr, int W, int H, int P, int num, int den, int origin)
{
    ColPlan c{};
    c.rows = skew_rows_plan(repr, H, W, P, num, den, origin);   // the transposed image has W lines of H pixels
    c.spread = c.rows.spread;
    const int Ht = H + (int)c.spread;
    if (repr == MORPH_PACKED) {
        c.t1 = r256(bitmap_bytes(H, (long long)W * P));
        c.t2 = r256(bitmap_bytes(Ht, (long long)W * P));
        c.tr = 0;
    } else {
        c.t1 = rle_bytes(H, (long long)W * P);
        c.t2 = rle_bytes(Ht, (long long)W * P);
        c.tr = r256(std::max(morph_transpose_rle_workspace_bytes(W, H, P),
                             morph_transpose_rle_workspace_bytes(Ht, W, P)));
    }
    c.total = c.t1 + c.t2 + std::max(c.rows.total, c.tr);
    return c;
}

int skew_cols_run(int repr, const void *dst, const void *src, int W, int H, int P, int num, int den, int origin,
                  int fill, char *ws, const ColPlan &c, hipStream_t s)
{
    const int Ht = H + (int)c.spread;
    char *scratch = ws + c.t1 + c.t2;
    int rc;
    if (repr == MORPH_PACKED) {
        const morph_bitmap_t T1{(uint64_t *)ws, H, W, (H + 63) / 64, P};
        const morph_bitmap_t T2{(uint64_t *)(ws + c.t1), Ht, W, (Ht + 63) / 64, P};
        rc = morph_transpose_packed(&T1, (const morph_bitmap_t *)src, (morph_stream_t)s);
        if (rc == MORPH_OK) rc = skew_rows_run(repr, &T2, &T1, H, W, P, num, den, origin, fill, scratch, c.rows, s);
        if (rc == MORPH_OK) rc = morph_transpose_packed((const morph_bitmap_t *)dst, &T2, (morph_stream_t)s);
        return rc;
    }
    const morph_rle_t T1 = rle_at(ws, H, W, P), T2 = rle_at(ws + c.t1, Ht, W, P);
    rc = morph_transpose_rle(&T1, (const morph_rle_t *)src, scratch, c.tr, (morph_stream_t)s);
    if (rc == MORPH_OK) rc = skew_rows_run(repr, &T2, &T1, H, W, P, num, den, origin, fill, scratch, c.rows, s);
    if (rc == MORPH_OK) rc = morph_transpose_rle((const morph_rle_t *)dst, &T2, scratch, c.tr, (morph_stream_t)s);
    return rc;
}

// ------------------------------------------------------------- rotation
// Three skews about the frame centre: along the lines by -tan(a/2), across
// them by sin(a), along them by -tan(a/2), each keeping every pixel.
constexpr int kRotDen = 1 << 16;
constexpr double kHalfPi = 1.5707963267948966 + 1e-12;   // rotations by at most a right angle

struct RotPlan {
    int t, sn, W1, H2, W3;
    SkewPlan s1, s3;
    ColPlan s2;
    size_t a1, a2, total;
};

bool rot_plan(int repr, int W, int H, int P, double angle, RotPlan &r)
{
    if (!std::isfinite(angle) || std::fabs(angle) > kHalfPi) return false;
    r.t = (int)std::llround(std::tan(angle / 2) * kRotDen);
    r.sn = (int)std::llround(std::sin(angle) * kRotDen);
    r.s1 = skew_rows_plan(repr, W, H, P, -r.t, kRotDen, H / 2);
    r.W1 = W + (int)r.s1.spread;
    r.s2 = skew_cols_plan(repr, r.W1, H, P, r.sn, kRotDen, r.W1 / 2);
    r.H2 = H + (int)r.s2.spread;
    r.s3 = skew_rows_plan(repr, r.W1, r.H2, P, -r.t, kRotDen, r.H2 / 2);
    r.W3 = r.W1 + (int)r.s3.spread;
    if (!dims_ok(r.W3, r.H2, P)) return false;
    if (repr == MORPH_PACKED) {
        r.a1 = r256(bitmap_bytes(r.W1, (long long)H * P));
        r.a2 = r256(bitmap_bytes(r.W1, (long long)r.H2 * P));
    } else {
        r.a1 = rle_bytes(r.W1, (long long)H * P);
        r.a2 = rle_bytes(r.W1, (long long)r.H2 * P);
    }
    r.total = r.a1 + r.a2 + std::max(std::max(r.s1.total, r.s3.total), r.s2.total);
    return true;
}

// ------------------------------------------------------------ line ops
// Erosion or dilation by a centred line of `length` pixels along the slope
// num/den (|num| <= den): shear the columns so that the line lies along
// the rows (column x moves by -floor(num x / den), plus an offset that
// keeps shifts non-negative), apply the horizontal operation, and shear
// back.  The columns are sheared as the lines of the transposed image.
struct LinePlan {
    long long off, Ht;
    size_t x1, x2, x3, x4, rect, sh, total;
};

bool line_plan(int repr, int op, int W, int H, int P, int length, int num, int den, LinePlan &l)
{
    if (den <= 0 || length < 1 || std::llabs((long long)num) > den) return false;
    long long vmax = 0, vmin = 0;
    // v(x) = -floor(num x / den) is monotone in x: its ends decide
    const long long vw = -floor_div((long long)num * (W - 1), den);
    vmin = std::min(0LL, vw);
    vmax = std::max(0LL, vw);
    l.off = -vmin;
    l.Ht = H + vmax + l.off;
    if (!dims_ok(l.Ht, W, P) || !dims_ok(W, l.Ht, P)) return false;
    const int Ht = (int)l.Ht;
    const morph_se_t se{length, 1, length / 2, 0};
    if (repr == MORPH_PACKED) {
        l.x1 = r256(bitmap_bytes(Ht, (long long)W * P));     // transposed source, then the result transposed
        l.x2 = l.x1;                                          // sheared, then sheared back
        l.x3 = r256(bitmap_bytes(W, (long long)Ht * P));     // the flat image
        l.x4 = l.x3;                                          // its operation
        l.rect = r256(morph_workspace_bytes(op, MORPH_PACKED, W, Ht * P, se));
    } else {
        l.x1 = rle_bytes(Ht, (long long)W * P);
        l.x2 = l.x1;
        l.x3 = rle_bytes(W, (long long)Ht * P);
        l.x4 = l.x3;
        l.rect = r256(std::max({morph_rle_workspace_bytes(op, W, Ht, P, se),
                                morph_transpose_rle_workspace_bytes(W, H, P),
                                morph_transpose_rle_workspace_bytes(W, Ht, P),
                                morph_transpose_rle_workspace_bytes(Ht, W, P),
                                morph_transpose_rle_workspace_bytes(H, W, P),
                                morph_shift_rows_rle_workspace_bytes(W * P)}));
    }
    l.sh = 2 * r256((size_t)W * P * 4);
    l.total = l.x1 + l.x2 + l.x3 + l.x4 + l.rect + l.sh;
    return true;
}

bool repr_ok(int repr) { return repr == MORPH_PACKED || repr == MORPH_RLE; }

int dims_of(int repr, const void *img, int &W, int &H, int &P)
{
    if (!img) return MORPH_E_INVAL;
    if (repr == MORPH_PACKED) {
        const morph_bitmap_t *b = (const morph_bitmap_t *)img;
        W = b->width; H = b->height; P = b->npages;
    } else {
        const morph_rle_t *r = (const morph_rle_t *)img;
        W = r->width; H = r->height; P = r->npages;
    }
    return dims_ok(W, H, P) ? MORPH_OK : MORPH_E_INVAL;
}

bool ws_ok(const void *ws, size_t ws_bytes, size_t need)
{
    return need == 0 || (ws && !(((uintptr_t)ws) & 255) && ws_bytes >= need);
}

int skew_entry(int repr, int axis, const void *dst, const void *src, int num, int den, int origin, int fill,
               void *ws, size_t ws_bytes, hipStream_t s)
{
    int W, H, P, dW, dH, dP;
    if (den <= 0 || (fill != 0 && fill != 1)) return MORPH_E_INVAL;
    int rc = dims_of(repr, src, W, H, P);
    if (rc != MORPH_OK) return rc;
    rc = dims_of(repr, dst, dW, dH, dP);
    if (rc != MORPH_OK) return rc;
    if (axis == 0) {
        const SkewPlan k = skew_rows_plan(repr, W, H, P, num, den, origin);
        if (dW != W + k.spread || dH != H || dP != P) return MORPH_E_SHAPE;
        if (!ws_ok(ws, ws_bytes, k.total)) return MORPH_E_WORKSPACE;
        return skew_rows_run(repr, dst, src, W, H, P, num, den, origin, fill, (char *)ws, k, s);
    }
    const ColPlan c = skew_cols_plan(repr, W, H, P, num, den, origin);
    if (dW != W || dH != H + c.spread || dP != P) return MORPH_E_SHAPE;
    if (!dims_ok(H + c.spread, W, P)) return MORPH_E_UNSUPPORTED;
    if (!ws_ok(ws, ws_bytes, c.total)) return MORPH_E_WORKSPACE;
    return skew_cols_run(repr, dst, src, W, H, P, num, den, origin, fill, (char *)ws, c, s);
}

int rotate_entry(int repr, const void *dst, const void *src, double angle, void *ws, size_t ws_bytes,
                 hipStream_t s)
{
    int W, H, P, dW, dH, dP;
    int rc = dims_of(repr, src, W, H, P);
    if (rc != MORPH_OK) return rc;
    rc = dims_of(repr, dst, dW, dH, dP);
    if (rc != MORPH_OK) return rc;
    RotPlan r{};
    if (!rot_plan(repr, W, H, P, angle, r)) return MORPH_E_UNSUPPORTED;
    if (dW != r.W3 || dH != r.H2 || dP != P) return MORPH_E_SHAPE;
    if (!ws_ok(ws, ws_bytes, r.total)) return MORPH_E_WORKSPACE;
    char *w = (char *)ws;
    char *scratch = w + r.a1 + r.a2;
    if (repr == MORPH_PACKED) {
        const morph_bitmap_t A1{(uint64_t *)w, r.W1, H, (r.W1 + 63) / 64, P};
        const morph_bitmap_t A2{(uint64_t *)(w + r.a1), r.W1, r.H2, (r.W1 + 63) / 64, P};
        rc = skew_rows_run(repr, &A1, src, W, H, P, -r.t, kRotDen, H / 2, 0, scratch, r.s1, s);
        if (rc == MORPH_OK)
            rc = skew_cols_run(repr, &A2, &A1, r.W1, H, P, r.sn, kRotDen, r.W1 / 2, 0, scratch, r.s2, s);
        if (rc == MORPH_OK)
            rc = skew_rows_run(repr, dst, &A2, r.W1, r.H2, P, -r.t, kRotDen, r.H2 / 2, 0, scratch, r.s3, s);
        return rc;
    }
    const morph_rle_t A1 = rle_at(w, r.W1, H, P), A2 = rle_at(w + r.a1, r.W1, r.H2, P);
    rc = skew_rows_run(repr, &A1, src, W, H, P, -r.t, kRotDen, H / 2, 0, scratch, r.s1, s);
    if (rc == MORPH_OK) rc = skew_cols_run(repr, &A2, &A1, r.W1, H, P, r.sn, kRotDen, r.W1 / 2, 0, scratch, r.s2, s);
    if (rc == MORPH_OK) rc = skew_rows_run(repr, dst, &A2, r.W1, r.H2, P, -r.t, kRotDen, r.H2 / 2, 0, scratch, r.s3, s);
    return rc;
}

int line_entry(int repr, int op, const void *dst, const void *src, int length, int num, int den, void *ws,
               size_t ws_bytes, hipStream_t s)
{
    if (op != MORPH_ERODE && op != MORPH_DILATE) return MORPH_E_INVAL;
    int W, H, P, dW, dH, dP;
    int rc = dims_of(repr, src, W, H, P);
    if (rc != MORPH_OK) return rc;
    rc = dims_of(repr, dst, dW, dH, dP);
    if (rc != MORPH_OK) return rc;
    if (dW != W || dH != H || dP != P) return MORPH_E_SHAPE;
    LinePlan l{};
    if (den <= 0 || length < 1 || std::llabs((long long)num) > den) return MORPH_E_INVAL;
    if (!line_plan(repr, op, W, H, P, length, num, den, l)) return MORPH_E_UNSUPPORTED;
    if (!ws_ok(ws, ws_bytes, l.total)) return MORPH_E_WORKSPACE;
    const int Ht = (int)l.Ht;
    const int fill = op == MORPH_ERODE ? 1 : 0;   // pixels brought in from outside take the border value
    const morph_se_t se{length, 1, length / 2, 0};
    char *w = (char *)ws;
    char *x1 = w, *x2 = x1 + l.x1, *x3 = x2 + l.x2, *x4 = x3 + l.x3, *rect = x4 + l.x4;
    int *fwd = (int *)(rect + l.rect), *back = (int *)(rect + l.rect + l.sh / 2);
    hipError_t e = fill_shifts(fwd, (long long)W * P, W, kShiftLineOut, num, den, 0, l.off, s);
    if (e == hipSuccess) e = fill_shifts(back, (long long)W * P, W, kShiftLineIn, num, den, 0, l.off, s);
    if (e != hipSuccess) { set_hip_error(e); return MORPH_E_HIP; }
    const morph_stream_t ms = (morph_stream_t)s;
    if (repr == MORPH_PACKED) {
        const morph_bitmap_t T{(uint64_t *)x1, H, W, (H + 63) / 64, P};           // W lines of H pixels
        const morph_bitmap_t S{(uint64_t *)x2, Ht, W, (Ht + 63) / 64, P};         // sheared
        const morph_bitmap_t F{(uint64_t *)x3, W, Ht, (W + 63) / 64, P};          // the line horizontal
        const morph_bitmap_t O{(uint64_t *)x4, W, Ht, (W + 63) / 64, P};          // operated
        const morph_bitmap_t T2{(uint64_t *)x1, Ht, W, (Ht + 63) / 64, P};        // operated, transposed
        const morph_bitmap_t B{(uint64_t *)x2, H, W, (H + 63) / 64, P};           // sheared back
        rc = morph_transpose_packed(&T, (const morph_bitmap_t *)src, ms);
        if (rc == MORPH_OK) rc = morph_shift_rows_packed(&S, &T, fwd, fill, ms);
        if (rc == MORPH_OK) rc = morph_transpose_packed(&F, &S, ms);
        if (rc == MORPH_OK) {
            rc = op == MORPH_ERODE ? morph_erode_rect_packed(&O, &F, se, l.rect ? rect : nullptr, l.rect, ms)
                                   : morph_dilate_rect_packed(&O, &F, se, l.rect ? rect : nullptr, l.rect, ms);
        }
        if (rc == MORPH_OK) rc = morph_transpose_packed(&T2, &O, ms);
        if (rc == MORPH_OK) rc = morph_shift_rows_packed(&B, &T2, back, 0, ms);
        if (rc == MORPH_OK) rc = morph_transpose_packed((const morph_bitmap_t *)dst, &B, ms);
        return rc;
    }
    const morph_rle_t T = rle_at(x1, H, W, P), S = rle_at(x2, Ht, W, P), F = rle_at(x3, W, Ht, P);
    const morph_rle_t O = rle_at(x4, W, Ht, P), T2 = rle_at(x1, Ht, W, P), B = rle_at(x2, H, W, P);
    rc = morph_transpose_rle(&T, (const morph_rle_t *)src, rect, l.rect, ms);
    if (rc == MORPH_OK) rc = morph_shift_rows_rle(&S, &T, fwd, fill, rect, l.rect, ms);
    if (rc == MORPH_OK) rc = morph_transpose_rle(&F, &S, rect, l.rect, ms);
    if (rc == MORPH_OK) {
        rc = op == MORPH_ERODE ? morph_erode_rect_rle(&O, &F, se, rect, l.rect, ms)
                               : morph_dilate_rect_rle(&O, &F, se, rect, l.rect, ms);
    }
    if (rc == MORPH_OK) rc = morph_transpose_rle(&T2, &O, rect, l.rect, ms);
    if (rc == MORPH_OK) rc = morph_shift_rows_rle(&B, &T2, back, 0, rect, l.rect, ms);
    if (rc == MORPH_OK) rc = morph_transpose_rle((const morph_rle_t *)dst, &B, rect, l.rect, ms);
    return rc;
}

// -------------------------------------------------------------- layout
// Layout analysis on runs (section "Connected Component Extraction and
// Statistics", and the page-layout use of section "Experiments"): the
// typical spacings are percentiles of the white runs between black ones,
// horizontally and (after a transpose) vertically; the pages are smeared
// by a rectangle of those sizes, and the components of the result are the
// blocks.  Workspace: horizontal histograms, the transposed runs and the
// transpose's scratch, vertical histograms, the percentile scratch and the
// two results, then the dilation's and the labelling's workspaces (the
// dilation's sized for the largest element the spacings allow).
struct LayoutPlan {
    size_t hb, hw, tr, tws, vb, vw, pct, g, dil, lab, total;
};

LayoutPlan layout_plan(int W, int H, int P, long long max_runs)
{
    LayoutPlan l{};
    l.hb = l.hw = r256((size_t)P * (W + 1) * 4);
    l.tr = rle_bytes(H, (long long)W * P);
    l.tws = r256(morph_transpose_rle_workspace_bytes(W, H, P));
    l.vb = l.vw = r256((size_t)P * (H + 1) * 4);
    l.pct = r256(std::max(morph_histogram_percentile_workspace_bytes(W + 1),
                          morph_histogram_percentile_workspace_bytes(H + 1)));
    l.g = 256;
    // the smear's element is known only once the spacings are read: the
    // workspace covers any element the band form of the dilation takes
    // (up to 384 rows; a taller one is refused after the read)
    const morph_se_t big{W + 1, 384, (W + 1) / 2, 192};
    l.dil = r256(morph_rle_workspace_bytes(MORPH_DILATE, W, H, P, big));
    l.lab = r256(morph_rle_label_workspace_bytes(H * P, max_runs));
    // the histograms and transposed runs are dead once the spacings are
    // read: the dilation and the labelling reuse their room
    const size_t first = l.hb + l.hw + l.tr + std::max(l.tws, l.vb + l.vw + l.pct);
    l.total = l.g + std::max(first, std::max(l.dil, l.lab));
    return l;
}

}  // namespace

}  // namespace morph

using namespace morph;

extern "C" {

int64_t morph_skew_spread(int32_t lines, int32_t num, int32_t den, int32_t origin)
{
    if (lines < 1 || den <= 0) return -1;
    long long vmin, spread;
    skew_range(lines, num, den, origin, vmin, spread);
    return spread;
}

size_t morph_skew_workspace_bytes(int repr, int axis, int32_t width, int32_t height, int32_t npages, int32_t num,
                                  int32_t den, int32_t origin)
{
    if (!repr_ok(repr) || (axis != 0 && axis != 1) || den <= 0 || !dims_ok(width, height, npages)) return 0;
    if (axis == 0) return skew_rows_plan(repr, width, height, npages, num, den, origin).total;
    return skew_cols_plan(repr, width, height, npages, num, den, origin).total;
}

int morph_skew_packed(int axis, const morph_bitmap_t *dst, const morph_bitmap_t *src, int32_t num, int32_t den,
                      int32_t origin, int32_t fill, void *ws, size_t ws_bytes, morph_stream_t stream)
{
    if (axis != 0 && axis != 1) return MORPH_E_INVAL;
    return skew_entry(MORPH_PACKED, axis, dst, src, num, den, origin, fill, ws, ws_bytes, (hipStream_t)stream);
}

int morph_skew_rle(int axis, const morph_rle_t *dst, const morph_rle_t *src, int32_t num, int32_t den,
                   int32_t origin, int32_t fill, void *ws, size_t ws_bytes, morph_stream_t stream)
{
    if (axis != 0 && axis != 1) return MORPH_E_INVAL;
    return skew_entry(MORPH_RLE, axis, dst, src, num, den, origin, fill, ws, ws_bytes, (hipStream_t)stream);
}

int morph_rotation_rationals(double angle, int32_t den, int32_t *tan_num, int32_t *sin_num)
{
    if (!tan_num || !sin_num || den < 1 || den > (1 << 24)) return MORPH_E_INVAL;
    if (!std::isfinite(angle) || std::fabs(angle) > kHalfPi) return MORPH_E_UNSUPPORTED;
    *tan_num = (int32_t)std::llround(std::tan(angle / 2) * den);
    *sin_num = (int32_t)std::llround(std::sin(angle) * den);
    return MORPH_OK;
}

int morph_rotate_dims(int32_t width, int32_t height, double angle, int32_t *out_width, int32_t *out_height)
{
    if (!out_width || !out_height || !dims_ok(width, height, 1)) return MORPH_E_INVAL;
    RotPlan r{};
    if (!rot_plan(MORPH_PACKED, width, height, 1, angle, r)) return MORPH_E_UNSUPPORTED;
    *out_width = r.W3;
    *out_height = r.H2;
    return MORPH_OK;
}

size_t morph_rotate_workspace_bytes(int repr, int32_t width, int32_t height, int32_t npages, double angle)
{
    RotPlan r{};
    if (!repr_ok(repr) || !dims_ok(width, height, npages) || !rot_plan(repr, width, height, npages, angle, r))
        return 0;
    return r.total;
}

int morph_rotate_packed(const morph_bitmap_t *dst, const morph_bitmap_t *src, double angle, void *ws,
                        size_t ws_bytes, morph_stream_t stream)
{
    return rotate_entry(MORPH_PACKED, dst, src, angle, ws, ws_bytes, (hipStream_t)stream);
}

int morph_rotate_rle(const morph_rle_t *dst, const morph_rle_t *src, double angle, void *ws, size_t ws_bytes,
                     morph_stream_t stream)
{
    return rotate_entry(MORPH_RLE, dst, src, angle, ws, ws_bytes, (hipStream_t)stream);
}

size_t morph_line_op_workspace_bytes(int repr, int op, int32_t width, int32_t height, int32_t npages,
                                     int32_t length, int32_t num, int32_t den)
{
    LinePlan l{};
    if (!repr_ok(repr) || (op != MORPH_ERODE && op != MORPH_DILATE) || !dims_ok(width, height, npages) ||
        !line_plan(repr, op, width, height, npages, length, num, den, l))
        return 0;
    return l.total;
}

int morph_line_op_packed(int op, const morph_bitmap_t *dst, const morph_bitmap_t *src, int32_t length, int32_t num,
                         int32_t den, void *ws, size_t ws_bytes, morph_stream_t stream)
{
    return line_entry(MORPH_PACKED, op, dst, src, length, num, den, ws, ws_bytes, (hipStream_t)stream);
}

int morph_line_op_rle(int op, const morph_rle_t *dst, const morph_rle_t *src, int32_t length, int32_t num,
                      int32_t den, void *ws, size_t ws_bytes, morph_stream_t stream)
{
    return line_entry(MORPH_RLE, op, dst, src, length, num, den, ws, ws_bytes, (hipStream_t)stream);
}

size_t morph_layout_rle_workspace_bytes(int32_t width, int32_t height, int32_t npages, int64_t max_runs)
{
    if (!dims_ok(width, height, npages) || max_runs < 0 || max_runs >= 0x7fffffffLL) return 0;
    return layout_plan(width, height, npages, max_runs).total;
}

int morph_layout_rle(const morph_rle_t *src, int32_t num, int32_t den, int32_t connectivity,
                     const morph_rle_t *smeared, int32_t *labels, int64_t max_runs, int32_t *comp_ptr,
                     morph_component_t *stats, int64_t max_components, int32_t *spacing, void *ws,
                     size_t ws_bytes, morph_stream_t stream)
{
    if (!src || !smeared || !spacing || num < 1 || den < num) return MORPH_E_INVAL;
    const int W = src->width, H = src->height, P = src->npages;
    if (!dims_ok(W, H, P)) return MORPH_E_INVAL;
    if (smeared->width != W || smeared->height != H || smeared->npages != P) return MORPH_E_SHAPE;
    if (max_runs < 0 || max_runs >= 0x7fffffffLL) return MORPH_E_INVAL;
    const LayoutPlan l = layout_plan(W, H, P, max_runs);
    if (!ws_ok(ws, ws_bytes, l.total)) return MORPH_E_WORKSPACE;
    const hipStream_t s = (hipStream_t)stream;
    const morph_stream_t ms = stream;
    char *w = (char *)ws;
    int32_t *g = (int32_t *)w;                 // the two spacings on the device
    char *a = w + l.g;
    int32_t *hb = (int32_t *)a, *hw = (int32_t *)(a + l.hb);
    const morph_rle_t T = rle_at(a + l.hb + l.hw, H, W, P);
    char *rest = a + l.hb + l.hw + l.tr;
    int32_t *vb = (int32_t *)rest, *vw = (int32_t *)(rest + l.vb);
    char *pct = rest + l.vb + l.vw;
    int rc = morph_rle_run_histograms(src, hb, hw, ms);
    if (rc == MORPH_OK) rc = morph_histogram_percentile(hw, P, W + 1, num, den, g, pct, l.pct, ms);
    if (rc == MORPH_OK) rc = morph_transpose_rle(&T, src, rest, l.tws, ms);
    if (rc == MORPH_OK) rc = morph_rle_run_histograms(&T, vb, vw, ms);
    if (rc == MORPH_OK) rc = morph_histogram_percentile(vw, P, H + 1, num, den, g + 1, pct, l.pct, ms);
    if (rc != MORPH_OK) return rc;
    int32_t host[2];
    hipError_t e = hipMemcpyAsync(host, g, sizeof(host), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) { set_hip_error(e); return MORPH_E_HIP; }
    spacing[0] = host[0];
    spacing[1] = host[1];
    const morph_se_t se{host[0] + 1, host[1] + 1, (host[0] + 1) / 2, (host[1] + 1) / 2};
    if (morph_rle_workspace_bytes(MORPH_DILATE, W, H, P, se) > l.dil) return MORPH_E_UNSUPPORTED;
    rc = morph_dilate_rect_rle(smeared, src, se, a, l.dil, ms);
    if (rc == MORPH_OK) rc = morph_rle_label(smeared, connectivity, labels, max_runs, comp_ptr, a, l.lab, ms);
    if (rc == MORPH_OK)
        rc = morph_rle_component_stats(smeared, labels, max_runs, comp_ptr, stats, max_components, ms);
    return rc;
}

}  // extern "C"
