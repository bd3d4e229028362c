// Run-length images on gfx950: conversion, within-line and between-line
// passes, and the device-wide scans they use.
//
// Layout: CSR over rows, runs as half-open int32 pairs [start, end).  Every
// kernel that produces runs works in two launches around a scan: a count
// launch writes the number of output runs of each row, an exclusive scan
// turns the counts into row offsets, and an emit launch recomputes the rows
// and writes the runs at their offsets.  No device memory is allocated; all
// intermediates live in the caller's workspace.
//
// Method (paper): a rectangle operation on a run-length image is done
// within lines first, then between lines (section "2D Morphological
// Operators for Rectangular Masks", third strategy, which the paper found
// fastest, with the within-line part first because it handles images with
// many runs more cheaply).  Within a line, erosion shrinks every run and
// drops the ones that vanish, dilation grows them and merges the ones that
// meet (section "Within-Line Morphological Operations").  Between lines,
// erosion is the intersection and dilation the union of the run lists of h
// consecutive lines, computed by the logarithmic decomposition (section
// "Efficient Binary Decompositions": doubling offsets 1, 2, 4, ... then one
// last offset h - m) where every step is an ordered merge of two lines'
// runs (section "Between Line Boolean Operations").
#include "common.h"

#include <algorithm>

namespace morph {

namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanBlock = kScanThreads * kScanItems;   // items per scan block
constexpr int kRowWaves = 4;                             // rows per workgroup (one wave each)

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63); }

// Inclusive prefix sum over the 64 lanes of a wave.
__device__ __forceinline__ int wave_incl_scan(int x)
{
    const int lane = lane_id();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int t = __shfl_up(x, d, 64);
        if (lane >= d) x += t;
    }
    return x;
}

// Exclusive prefix sum over a workgroup of kScanThreads threads; *total
// receives the sum of all values.
__device__ __forceinline__ int block_excl_scan(int x, int *smem, int *total)
{
    const int lane = lane_id(), wave = threadIdx.x >> 6;
    const int inc = wave_incl_scan(x);
    if (lane == 63) smem[wave] = inc;
    __syncthreads();
    int wbase = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < kScanThreads / 64; k++) {
        const int v = smem[k];
        if (k < wave) wbase += v;
        tot += v;
    }
    __syncthreads();
    *total = tot;
    return wbase + inc - x;
}

// ------------------------------------------------------------------- scans
__global__ __launch_bounds__(kScanThreads) void scan_up_kernel(const int *__restrict__ in, int n,
                                                               int *__restrict__ bsum)
{
    __shared__ int smem[kScanThreads / 64];
    const long long base = (long long)blockIdx.x * kScanBlock + (long long)threadIdx.x * kScanItems;
    int s = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; i++)
        if (base + i < n) s += in[base + i];
    int tot;
    block_excl_scan(s, smem, &tot);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

// Exclusive scan of the block sums, in place, by one workgroup.
__global__ __launch_bounds__(kScanThreads) void scan_mid_kernel(int *bsum, int nb)
{
    __shared__ int smem[kScanThreads / 64];
    int carry = 0;
    for (int b0 = 0; b0 < nb; b0 += kScanThreads) {
        const int i = b0 + (int)threadIdx.x;
        const int v = i < nb ? bsum[i] : 0;
        int tot;
        const int ex = block_excl_scan(v, smem, &tot);
        if (i < nb) bsum[i] = carry + ex;
        carry += tot;
    }
}

__global__ __launch_bounds__(kScanThreads) void scan_down_kernel(const int *__restrict__ in, int n,
                                                                 const int *__restrict__ bsum,
                                                                 int *__restrict__ out)
{
    __shared__ int smem[kScanThreads / 64];
    const long long base = (long long)blockIdx.x * kScanBlock + (long long)threadIdx.x * kScanItems;
    int v[kScanItems];
    int s = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; i++) {
        v[i] = (base + i < n) ? in[base + i] : 0;
        s += v[i];
    }
    int tot;
    int run = block_excl_scan(s, smem, &tot) + bsum[blockIdx.x];
#pragma unroll
    for (int i = 0; i < kScanItems; i++) {
        if (base + i < n) out[base + i] = run;
        run += v[i];
    }
    // the thread holding the last item also writes the grand total
    if (base < n && base + kScanItems >= n) out[n] = run;
}

__global__ void zero_one_kernel(int *out)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) out[0] = 0;
}

// -------------------------------------------------------- packed -> runs
// One wave per row.  For each word a: a start is a 1 whose left neighbour
// is 0 (or the left border), an end is a 0 whose left neighbour is 1; the
// pad bits are 0, and a virtual zero word after the row gives the end at
// the right border when the width is a multiple of 64.
template <bool EMIT>
__global__ __launch_bounds__(64 * kRowWaves) void pack_to_rle_kernel(
    const uint64_t *__restrict__ words, int nw, int stride, int H, int R, long long page_words,
    uint64_t padmask, int *__restrict__ counts, const int *__restrict__ row_ptr,
    int *__restrict__ runs, long long cap)
{
    const int r = blockIdx.x * kRowWaves + (int)(threadIdx.x >> 6);
    if (r >= R) return;                    // whole wave
    const int lane = lane_id();
    const int page = r / H, y = r - page * H;
    const uint64_t *row = words + (long long)page * page_words + (long long)y * stride;
    long long obase = EMIT ? row_ptr[r] : 0;
    int cstart = 0, cend = 0;
    uint64_t prev = 0;                     // bit 63 of the previous chunk's last word
    for (int j0 = 0; j0 <= nw; j0 += 64) {
        const int j = j0 + lane;
        uint64_t a = 0;
        if (j < nw) {
            a = row[j];
            if (j == nw - 1) a &= padmask;
        }
        uint64_t up = (uint64_t)__shfl_up((int)(a >> 63), 1, 64);
        if (lane == 0) up = prev;
        const uint64_t sh = (a << 1) | up;
        uint64_t st = a & ~sh, en = ~a & sh;
        if (j > nw) { st = 0; en = 0; }
        const int ns = __popcll(st), ne = __popcll(en);
        const int is = wave_incl_scan(ns), ie = wave_incl_scan(ne);
        if (EMIT) {
            long long k = obase + cstart + is - ns;
            while (st) {
                const int b = __ffsll((unsigned long long)st) - 1;
                if (k < cap) runs[2 * k] = 64 * j + b;
                k++;
                st &= st - 1;
            }
            k = obase + cend + ie - ne;
            while (en) {
                const int b = __ffsll((unsigned long long)en) - 1;
                if (k < cap) runs[2 * k + 1] = 64 * j + b;
                k++;
                en &= en - 1;
            }
        }
        cstart += __shfl(is, 63, 64);
        cend += __shfl(ie, 63, 64);
        prev = (uint64_t)__shfl((int)(a >> 63), 63, 64);
    }
    if (!EMIT && lane == 0) counts[r] = cstart;
}

// -------------------------------------------------------- runs -> packed
// One thread per output word: binary search for the first run ending after
// the word's first pixel, then OR in every run that starts before its end.
__global__ __launch_bounds__(256) void rle_to_pack_kernel(const int *__restrict__ row_ptr,
                                                          const int *__restrict__ runs, int nw,
                                                          int R, int H, uint64_t *__restrict__ words,
                                                          int stride, long long page_words)
{
    const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
    if (t >= (long long)R * nw) return;
    const int r = (int)(t / nw), j = (int)(t - (long long)r * nw);
    const int page = r / H, y = r - page * H;
    int lo = row_ptr[r];
    int hi = row_ptr[r + 1];
    const int x0 = 64 * j, x1 = x0 + 64;
    while (lo < hi) {                      // first run with end > x0
        const int mid = (lo + hi) >> 1;
        if (runs[2 * mid + 1] > x0) hi = mid; else lo = mid + 1;
    }
    uint64_t v = 0;
    const int end = row_ptr[r + 1];
    for (int k = lo; k < end; k++) {
        const int s = runs[2 * k], e = runs[2 * k + 1];
        if (s >= x1) break;
        const int a = max(s, x0) - x0, b = min(e, x1) - x0;   // 0 <= a < b <= 64
        const uint64_t hiMask = (b == 64) ? ~0ull : ((1ull << b) - 1);
        v |= hiMask & ~((1ull << a) - 1);
    }
    words[(long long)page * page_words + (long long)y * stride + j] = v;
}

// ------------------------------------------------------ within-line pass
// One wave per row, lanes over runs.  Erosion by a 1 x w element with
// origin cx: [s, e) -> [s + cx, e - (w-1-cx)), a side on the row border
// stays where it is (outside pixels are 1), and empty runs are dropped.
// Dilation: [s, e) -> [s - cx, e + w-1-cx) clipped to [0, W), and runs that
// overlap or touch are merged.
template <bool EMIT, bool DILATE>
__global__ __launch_bounds__(64 * kRowWaves) void row_pass_kernel(
    const int *__restrict__ in_rp, const int *__restrict__ in_runs, long long in_cap, int R, int W,
    int w, int cx, int *__restrict__ counts, const int *__restrict__ out_rp,
    int *__restrict__ out_runs, long long out_cap)
{
    const int r = blockIdx.x * kRowWaves + (int)(threadIdx.x >> 6);
    if (r >= R) return;
    const int lane = lane_id();
    // a malformed row_ptr cannot send reads past the input's capacity
    const int b0 = (int)min((long long)max(in_rp[r], 0), in_cap);
    const int n = (int)max(0LL, min((long long)in_rp[r + 1], in_cap) - b0);
    const int left = DILATE ? cx : -cx;                 // start moves to s - left
    const int right = DILATE ? (w - 1 - cx) : -(w - 1 - cx);
    const unsigned long long lt = (1ull << lane) - 1;
    long long obase = EMIT ? out_rp[r] : 0;
    int carry = 0;
    for (int k0 = 0; k0 < n; k0 += 64) {
        const int k = k0 + lane;
        const bool valid = k < n;
        int s = 0, e = 0;
        if (valid) {
            s = in_runs[2 * (b0 + k)];
            e = in_runs[2 * (b0 + k) + 1];
        }
        int ns, ne;
        if (DILATE) {
            ns = max(0, s - left);
            ne = min(W, e + right);
        } else {
            ns = (s == 0) ? 0 : s - left;
            ne = (e == W) ? W : e + right;
        }
        bool first, last;
        if (DILATE) {
            // a run starts a group unless it meets the previous run's grown end
            int pe = -1;
            if (valid && k > 0) pe = min(W, in_runs[2 * (b0 + k - 1) + 1] + right);
            first = valid && (k == 0 || ns > pe);
            last = valid && (k == n - 1 || max(0, in_runs[2 * (b0 + k + 1)] - left) > ne);
        } else {
            first = last = valid && ns < ne;
        }
        const unsigned long long fm = __ballot(first);
        const int idx = carry + __popcll(fm & lt);
        if (EMIT) {
            const long long o = obase + idx;
            if (first && o < out_cap) out_runs[2 * o] = ns;
            const long long oe = o - (first ? 0 : 1);
            if (last && oe >= 0 && oe < out_cap) out_runs[2 * oe + 1] = ne;
        }
        carry += __popcll(fm);
    }
    if (!EMIT && lane == 0) counts[r] = carry;
}

// ----------------------------------------------------- between-line pass
// A view of a run-length image with virtual rows: row r of page p is real
// row r - off of that page if it lies in [0, real), otherwise it is the
// full row [0, W) (erosion) or the empty row (dilation).
struct RowView {
    const int *rp;
    const int *runs;
    long long cap;            // runs the runs array holds
    int off, real, rows;      // rows = rows per page seen through the view
};

struct Row {
    const int *runs;
    int n;
    bool full;
};

__device__ __forceinline__ Row view_row(const RowView &v, int page, int r, bool erode)
{
    const int rr = r - v.off;
    Row o;
    if (rr >= 0 && rr < v.real) {
        const int i = page * v.real + rr;
        const long long b = min((long long)max(v.rp[i], 0), v.cap);
        o.runs = v.runs + 2 * b;
        o.n = (int)max(0LL, min((long long)v.rp[i + 1], v.cap) - b);
        o.full = false;
    } else {
        o.runs = nullptr;
        o.n = erode ? 1 : 0;
        o.full = true;
    }
    return o;
}

__device__ __forceinline__ void run_at(const Row &r, int k, int W, int &s, int &e)
{
    if (r.full) { s = 0; e = W; }
    else { s = r.runs[2 * k]; e = r.runs[2 * k + 1]; }
}

// One thread per output row: out[r] = A[r] AND A[r+K] (erosion) or
// A[r] OR A[r+K] (dilation), as an ordered merge of the two run lists.
template <bool EMIT, bool ERODE>
__global__ __launch_bounds__(256) void col_stage_kernel(RowView A, int K, int P, int W,
                                                        int *__restrict__ counts,
                                                        const int *__restrict__ out_rp,
                                                        int *__restrict__ out_runs, long long out_cap)
{
    const int NB = A.rows - K;
    const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
    if (t >= (long long)P * NB) return;
    const int page = (int)(t / NB), r = (int)(t - (long long)page * NB);
    const Row a = view_row(A, page, r, ERODE), b = view_row(A, page, r + K, ERODE);
    long long o = EMIT ? out_rp[t] : 0;
    int cnt = 0;
    int i = 0, j = 0;
    if (ERODE) {
        while (i < a.n && j < b.n) {
            int as, ae, bs, be;
            run_at(a, i, W, as, ae);
            run_at(b, j, W, bs, be);
            const int s = max(as, bs), e = min(ae, be);
            if (s < e) {
                if (EMIT) { if (o < out_cap) { out_runs[2 * o] = s; out_runs[2 * o + 1] = e; } o++; }
                cnt++;
            }
            if (ae <= be) i++;
            if (be <= ae) j++;
        }
    } else {
        int cs = 0, ce = -1;               // current merged run, none yet
        while (i < a.n || j < b.n) {
            int s, e;
            int as = 0x7fffffff, ae = 0, bs = 0x7fffffff, be = 0;
            if (i < a.n) run_at(a, i, W, as, ae);
            if (j < b.n) run_at(b, j, W, bs, be);
            if (as <= bs) { s = as; e = ae; i++; } else { s = bs; e = be; j++; }
            if (ce >= 0 && s <= ce) {
                ce = max(ce, e);
            } else {
                if (ce >= 0) {
                    if (EMIT) { if (o < out_cap) { out_runs[2 * o] = cs; out_runs[2 * o + 1] = ce; } o++; }
                    cnt++;
                }
                cs = s;
                ce = e;
            }
        }
        if (ce >= 0) {
            if (EMIT) { if (o < out_cap) { out_runs[2 * o] = cs; out_runs[2 * o + 1] = ce; } o++; }
            cnt++;
        }
    }
    if (!EMIT) counts[t] = cnt;
}

// Canonical-form check: sets *bad when a row breaks it.
__global__ __launch_bounds__(256) void validate_kernel(const int *__restrict__ rp,
                                                       const int *__restrict__ runs, int R, int W,
                                                       long long cap, int *bad)
{
    const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
    if (t >= R) return;
    const int b = rp[t], e = rp[t + 1];
    bool ok = b >= 0 && (t > 0 || b == 0) && b <= e && (long long)e <= cap;
    int last = -1;
    for (int k = b; ok && k < e; k++) {
        const int s = runs[2 * k], f = runs[2 * k + 1];
        if (!(s > last && s < f && f <= W && s >= 0)) ok = false;
        last = f;
    }
    if (!ok) atomicOr(bad, 1);
}

unsigned blocks_for(long long n, int per) { return (unsigned)((n + per - 1) / per); }

}  // namespace

// --------------------------------------------------------- host helpers
size_t scan_workspace(int64_t n) { return (size_t)((n + kScanBlock - 1) / kScanBlock + 1) * sizeof(int); }

// out[0..n] = exclusive scan of in[0..n-1], out[n] = total.
static hipError_t exclusive_scan(const int *in, int n, int *out, int *tmp, hipStream_t s)
{
    if (n == 0) {
        hipLaunchKernelGGL(zero_one_kernel, dim3(1), dim3(64), 0, s, out);
        return hipGetLastError();
    }
    const unsigned nb = blocks_for(n, kScanBlock);
    hipLaunchKernelGGL(scan_up_kernel, dim3(nb), dim3(kScanThreads), 0, s, in, n, tmp);
    hipLaunchKernelGGL(scan_mid_kernel, dim3(1), dim3(kScanThreads), 0, s, tmp, (int)nb);
    hipLaunchKernelGGL(scan_down_kernel, dim3(nb), dim3(kScanThreads), 0, s, in, n, tmp, out);
    return hipGetLastError();
}

static size_t r256(size_t b) { return (b + 255) & ~(size_t)255; }

hipError_t rle_from_packed(const morph_rle_t &dst, const morph_bitmap_t &src, void *ws, hipStream_t s)
{
    const int R = src.height * src.npages;
    const int nw = (src.width + 63) / 64;
    const uint64_t pad = (src.width % 64) ? ((1ull << (src.width % 64)) - 1) : ~0ull;
    int *counts = (int *)ws;
    int *tmp = (int *)((char *)ws + r256((size_t)R * sizeof(int)));
    const long long pw = (long long)src.stride_words * src.height;
    const unsigned g = blocks_for(R, kRowWaves);
    hipLaunchKernelGGL((pack_to_rle_kernel<false>), dim3(g), dim3(64 * kRowWaves), 0, s, src.words, nw,
                       src.stride_words, src.height, R, pw, pad, counts, nullptr, nullptr, 0LL);
    hipError_t e = exclusive_scan(counts, R, dst.row_ptr, tmp, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((pack_to_rle_kernel<true>), dim3(g), dim3(64 * kRowWaves), 0, s, src.words, nw,
                       src.stride_words, src.height, R, pw, pad, nullptr, dst.row_ptr, dst.runs,
                       (long long)dst.capacity);
    return hipGetLastError();
}

hipError_t rle_to_packed(const morph_bitmap_t &dst, const morph_rle_t &src, hipStream_t s)
{
    const int R = src.height * src.npages;
    const int nw = (src.width + 63) / 64;
    const long long total = (long long)R * nw;
    hipLaunchKernelGGL(rle_to_pack_kernel, dim3(blocks_for(total, 256)), dim3(256), 0, s, src.row_ptr,
                       src.runs, nw, R, src.height, dst.words, dst.stride_words,
                       (long long)dst.stride_words * dst.height);
    return hipGetLastError();
}

// Workspace layout of a run-length rectangle operation on P pages of H rows:
//   counts[P*(H+h-1)] | scan tmp | T0 (row pass out) | T1, T2 (stages) | T3 (open/close middle)
struct RleWs {
    int *counts, *tmp;
    int *rp[4];
    int *runs[4];
    size_t bytes;
};

static RleWs rle_layout(void *base, int op, int32_t W, int32_t rows, int32_t H, morph_se_t se)
{
    const int P = rows / H;
    const long long ext = (long long)P * (H + se.h - 1);
    const long long half = (W + 1) / 2;
    RleWs L{};
    char *p = (char *)base;
    size_t off = 0;
    auto take = [&](size_t b) { char *q = p ? p + off : nullptr; off += r256(b); return (int *)q; };
    L.counts = take((size_t)ext * 4);
    L.tmp = take(scan_workspace(ext));
    const long long rows_of[4] = {(long long)P * H, ext, ext, (long long)P * H};
    const int nbuf = (op == MORPH_OPEN || op == MORPH_CLOSE) ? 4 : 3;
    for (int i = 0; i < 4; i++) {
        if (i < nbuf) {
            L.rp[i] = take((size_t)(rows_of[i] + 1) * 4);
            L.runs[i] = take((size_t)rows_of[i] * half * 8);
        } else {
            L.rp[i] = nullptr;
            L.runs[i] = nullptr;
        }
    }
    L.bytes = off;
    return L;
}

size_t rle_op_workspace(int op, int32_t W, int32_t rows, int32_t H, morph_se_t se)
{
    return rle_layout(nullptr, op, W, rows, H, se).bytes;
}

// One erosion or dilation of P pages: src (CSR) -> dst (CSR).
static hipError_t rle_erode_dilate(bool erode, const int *src_rp, const int *src_runs,
                                   long long src_cap, int *dst_rp, int *dst_runs, long long dst_cap,
                                   int P, int W, int H, morph_se_t se, const RleWs &L, hipStream_t s)
{
    const int R = P * H;
    const long long half = (W + 1) / 2;
    const unsigned g = blocks_for(R, kRowWaves);
    // within-line pass; skipped when the element is one pixel wide, unless
    // nothing else runs (then it copies src to dst)
    const bool rowpass = se.w > 1 || se.h == 1;
    const int *cur_rp = src_rp, *cur_runs = src_runs;
    long long cur_cap = src_cap;
    if (rowpass) {
        int *o_rp = se.h == 1 ? dst_rp : L.rp[0];
        int *o_runs = se.h == 1 ? dst_runs : L.runs[0];
        const long long o_cap = se.h == 1 ? dst_cap : (long long)R * half;
        if (erode) {
            hipLaunchKernelGGL((row_pass_kernel<false, false>), dim3(g), dim3(64 * kRowWaves), 0, s, src_rp,
                               src_runs, src_cap, R, W, se.w, se.cx, L.counts, nullptr, nullptr, 0LL);
        } else {
            hipLaunchKernelGGL((row_pass_kernel<false, true>), dim3(g), dim3(64 * kRowWaves), 0, s, src_rp,
                               src_runs, src_cap, R, W, se.w, se.cx, L.counts, nullptr, nullptr, 0LL);
        }
        hipError_t e = exclusive_scan(L.counts, R, o_rp, L.tmp, s);
        if (e != hipSuccess) return e;
        if (erode) {
            hipLaunchKernelGGL((row_pass_kernel<true, false>), dim3(g), dim3(64 * kRowWaves), 0, s, src_rp,
                               src_runs, src_cap, R, W, se.w, se.cx, nullptr, o_rp, o_runs, o_cap);
        } else {
            hipLaunchKernelGGL((row_pass_kernel<true, true>), dim3(g), dim3(64 * kRowWaves), 0, s, src_rp,
                               src_runs, src_cap, R, W, se.w, se.cx, nullptr, o_rp, o_runs, o_cap);
        }
        if ((e = hipGetLastError()) != hipSuccess) return e;
        cur_rp = o_rp;
        cur_runs = o_runs;
        cur_cap = o_cap;
    }
    if (se.h == 1) return hipSuccess;
    // between-line pass: rows of the extended page are r = 0 .. H+h-2, row r
    // being image row r - top (top = cy for erosion, h-1-cy for dilation)
    const int top = erode ? se.cy : se.h - 1 - se.cy;
    RowView v{cur_rp, cur_runs, cur_cap, top, H, H + se.h - 1};
    // offsets: 1, 2, 4, ... while doubling stays <= h, then h - m
    int offs[40], nst = 0;
    int m = 1;
    while (2 * m <= se.h) { offs[nst++] = m; m *= 2; }
    if (se.h > m) offs[nst++] = se.h - m;
    int ping = 1;
    for (int k = 0; k < nst; k++) {
        const int K = offs[k];
        const int NB = v.rows - K;
        const bool lastst = k + 1 == nst;
        int *o_rp = lastst ? dst_rp : L.rp[ping];
        int *o_runs = lastst ? dst_runs : L.runs[ping];
        const long long n = (long long)P * NB;
        const long long o_cap = lastst ? dst_cap : n * half;
        const unsigned gb = blocks_for(n, 256);
        if (erode)
            hipLaunchKernelGGL((col_stage_kernel<false, true>), dim3(gb), dim3(256), 0, s, v, K, P, W,
                               L.counts, nullptr, nullptr, 0LL);
        else
            hipLaunchKernelGGL((col_stage_kernel<false, false>), dim3(gb), dim3(256), 0, s, v, K, P, W,
                               L.counts, nullptr, nullptr, 0LL);
        hipError_t e = exclusive_scan(L.counts, (int)n, o_rp, L.tmp, s);
        if (e != hipSuccess) return e;
        if (erode)
            hipLaunchKernelGGL((col_stage_kernel<true, true>), dim3(gb), dim3(256), 0, s, v, K, P, W,
                               nullptr, o_rp, o_runs, o_cap);
        else
            hipLaunchKernelGGL((col_stage_kernel<true, false>), dim3(gb), dim3(256), 0, s, v, K, P, W,
                               nullptr, o_rp, o_runs, o_cap);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        v = RowView{o_rp, o_runs, o_cap, 0, NB, NB};
        ping = 3 - ping;
    }
    return hipSuccess;
}

hipError_t rle_rect_op(int op, const morph_rle_t &dst, const morph_rle_t &src, morph_se_t se,
                       void *ws, size_t ws_bytes, hipStream_t s)
{
    (void)ws_bytes;
    const int P = src.npages, H = src.height, W = src.width;
    const RleWs L = rle_layout(ws, op, W, P * H, H, se);
    switch (op) {
    case MORPH_ERODE:
    case MORPH_DILATE:
        return rle_erode_dilate(op == MORPH_ERODE, src.row_ptr, src.runs, src.capacity, dst.row_ptr,
                                dst.runs, dst.capacity, P, W, H, se, L, s);
    case MORPH_OPEN:
    case MORPH_CLOSE: {
        const bool e1 = op == MORPH_OPEN;
        const long long mid_cap = (long long)P * H * ((W + 1) / 2);
        hipError_t e = rle_erode_dilate(e1, src.row_ptr, src.runs, src.capacity, L.rp[3], L.runs[3],
                                        mid_cap, P, W, H, se, L, s);
        if (e != hipSuccess) return e;
        return rle_erode_dilate(!e1, L.rp[3], L.runs[3], mid_cap, dst.row_ptr, dst.runs, dst.capacity,
                                P, W, H, se, L, s);
    }
    }
    return hipErrorInvalidValue;
}

int rle_validate(const morph_rle_t &r, hipStream_t s, hipError_t *err)
{
    const int R = r.height * r.npages;
    int *flag = nullptr;
    hipError_t e = hipMalloc(&flag, sizeof(int));
    if (e == hipSuccess) e = hipMemsetAsync(flag, 0, sizeof(int), s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(validate_kernel, dim3(blocks_for(R, 256)), dim3(256), 0, s, r.row_ptr, r.runs, R,
                           r.width, (long long)r.capacity, flag);
        e = hipGetLastError();
    }
    int host = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&host, flag, sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (flag) hipFree(flag);
    *err = e;
    if (e != hipSuccess) return MORPH_E_HIP;
    return host ? MORPH_E_NONCANONICAL : MORPH_OK;
}

}  // namespace morph
