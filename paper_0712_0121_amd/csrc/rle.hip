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
#include <mutex>

namespace morph {

namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanBlock = kScanThreads * kScanItems;   // items per scan block
constexpr int kRowWaves = 4;                             // rows per workgroup (one wave each)

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63); }

// Trace counters: runs read / written, spread over 256 slots (one 128-byte
// line each) so that concurrent groups rarely add to the same address.
constexpr int kTraceSlots = 256, kTraceStride = 16;

__device__ __forceinline__ void trace_add(unsigned long long *tr, unsigned long long in, unsigned long long out)
{
    const int slot = (int)((blockIdx.x * 16u + (threadIdx.x >> 4)) & (kTraceSlots - 1));
    if (in) atomicAdd(tr + (long long)slot * kTraceStride, in);
    if (out) atomicAdd(tr + (long long)(kTraceSlots + slot) * kTraceStride, out);
}


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

// The whole scan in one workgroup for short inputs (a page's rows): blocks
// of kScanBlock in turn with a carry, the grand total at out[n].  One launch
// instead of three, which is most of the scan's time on a single page.
constexpr int kScanSingleMax = 4 * kScanBlock;

__global__ __launch_bounds__(kScanThreads) void scan_single_kernel(const int *__restrict__ in, int n,
                                                                   int *__restrict__ out)
{
    __shared__ int smem[kScanThreads / 64];
    int carry = 0;
    for (int b0 = 0; b0 < n; b0 += kScanBlock) {
        const int base = b0 + (int)threadIdx.x * kScanItems;
        int v[kScanItems];
        int s = 0;
#pragma unroll
        for (int i = 0; i < kScanItems; i++) {
            v[i] = (base + i < n) ? in[base + i] : 0;
            s += v[i];
        }
        int tot;
        int run = block_excl_scan(s, smem, &tot) + carry;
#pragma unroll
        for (int i = 0; i < kScanItems; i++) {
            if (base + i < n) out[base + i] = run;
            run += v[i];
        }
        carry += tot;
    }
    if (threadIdx.x == 0) out[n] = carry;
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

// Writes every run that ends in this lane's word as one pair at k, k + 1,
// ...: the word covers pixels base .. base + 63, st and en are its start and
// end bits (an end at bit b: pixel b is white, pixel b - 1 black), and a
// run whose start is not in the word started at `before` (the last start
// of an earlier word; runs alternate with gaps).  Works on the two 32-bit
// halves, one end per step.
__device__ __forceinline__ void emit_word_runs(uint64_t st, uint64_t en, int base, int before, int k, int cap,
                                               int *__restrict__ runs)
{
    const uint32_t st_lo = (uint32_t)st, st_hi = (uint32_t)(st >> 32);
    uint32_t en_lo = (uint32_t)en, en_hi = (uint32_t)(en >> 32);
    // the last start of the low half (or the start before the word)
    const int ls_lo = st_lo ? base + 31 - (int)__clz(st_lo) : before;
    while (en_lo | en_hi) {
        const bool lo = en_lo != 0;
        const uint32_t e = lo ? en_lo : en_hi;
        const int b = __ffs(e) - 1;
        const uint32_t below = (lo ? st_lo : st_hi) & ((1u << b) - 1u);
        const int half = lo ? base : base + 32;
        const int s0 = below ? half + 31 - (int)__clz(below) : (lo ? before : ls_lo);
        if (k < cap) reinterpret_cast<int2 *>(runs)[k] = make_int2(s0, half + b);
        k++;
        if (lo) en_lo = e & (e - 1u); else en_hi = e & (e - 1u);
    }
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
    int *__restrict__ runs, long long cap, unsigned long long *trace)
{
    const int r = blockIdx.x * kRowWaves + (int)(threadIdx.x >> 6);
    if (r >= R) return;                    // whole wave
    const int lane = lane_id();
    const int page = r / H, y = r - page * H;
    const uint64_t *row = words + (long long)page * page_words + (long long)y * stride;
    long long obase = EMIT ? row_ptr[r] : 0;
    const int capi = (int)min(cap, 0x7fffffffLL);   // run indices fit in int: row offsets are int
    int cstart = 0, cend = 0;
    uint64_t prev = 0;                     // bit 63 of the previous chunk's last word
    int last_start = -1;                   // the last start before this chunk (-1: none)
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
        const int ns = EMIT ? 0 : __popcll(st), ne = EMIT ? __popcll(en) : 0;
        const int is = EMIT ? 0 : wave_incl_scan(ns), ie = EMIT ? wave_incl_scan(ne) : 0;
        if (EMIT) {
            // each run written whole by the lane of its end (see the
            // grouped kernel below)
            int incl = st ? 64 * j + 63 - (int)__clzll(st) : -1;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const int y = __shfl_up(incl, o, 64);
                if (lane >= o) incl = max(incl, y);
            }
            int before = __shfl_up(incl, 1, 64);
            before = lane == 0 ? last_start : max(last_start, before);
            emit_word_runs(st, en, 64 * j, before, (int)(obase + cend + ie - ne), capi, runs);
            last_start = max(last_start, __shfl(incl, 63, 64));
        }
        if (EMIT) cend += __shfl(ie, 63, 64); else cstart += __shfl(is, 63, 64);
        prev = (uint64_t)__shfl((int)(a >> 63), 63, 64);
    }
    if (!EMIT && lane == 0) counts[r] = cstart;
    if (EMIT && trace && lane == 0) trace_add(trace, 0, (unsigned long long)cend);
}

// -------------------------------------------------------- runs -> packed
// One thread per output word: binary search for the first run ending after
// the word's first pixel, then OR in every run that starts before its end.
// The host launches it only while rows x words stays below 2^32.
__global__ __launch_bounds__(256) void rle_to_pack_kernel(const int *__restrict__ row_ptr,
                                                          const int *__restrict__ runs, int nw,
                                                          int R, int H, uint64_t *__restrict__ words,
                                                          int stride, long long page_words, long long cap,
                                                          unsigned long long *trace)
{
    const unsigned t = blockIdx.x * 256u + threadIdx.x;
    if (t >= (unsigned)R * (unsigned)nw) return;
    const int r = (int)(t / (unsigned)nw), j = (int)(t - (unsigned)r * (unsigned)nw);
    const int page = r / H, y = r - page * H;
    // offsets clamped to the run array, so a damaged row_ptr cannot send
    // the reads outside it
    const int b0 = (int)min((long long)max(row_ptr[r], 0), cap);
    const int b1 = (int)max((long long)b0, min((long long)row_ptr[r + 1], cap));
    const int x0 = 64 * j, x1 = x0 + 64;
    int lo = b0, hi = b1;
    while (lo < hi) {                      // first run with end > x0
        const int mid = (lo + hi) >> 1;
        if (runs[2 * mid + 1] > x0) hi = mid; else lo = mid + 1;
    }
    uint64_t v = 0;
    for (int k = lo; k < b1; k++) {
        const int s = runs[2 * k], e = runs[2 * k + 1];
        if (s >= x1) break;
        const int a = max(s, x0) - x0, b = min(e, x1) - x0;   // 0 <= a < b <= 64
        const uint64_t hiMask = (b == 64) ? ~0ull : ((1ull << b) - 1);
        v |= hiMask & ~((1ull << a) - 1);
    }
    words[(long long)page * page_words + (long long)y * stride + j] = v;
    if (trace && j == 0) trace_add(trace, (unsigned long long)(b1 - b0), 0);
}

// ------------------------------------------ runs -> transposed packed
// One workgroup of kDecodeWaves waves per group of kDecodeWaves 64-row
// blocks and strip of kDecodeStrip words.  Lane i of wave q streams the
// runs of row 64(k0 + q) + i once, in order (one 8-byte load per run),
// turns each run -- or each gap, for a complemented operation -- into an
// interval by the row's within-line operation, and ORs the intervals into
// the word being built; an interval that reaches past the word is kept in
// registers for the next one.  The operation moves starts and ends
// monotonically, so once an interval reaches past the word every later
// one's part of the word lies inside it.  For every word the butterfly
// turns the 64 x 64 block; the transposed words wait in LDS until the
// workgroup has all of them, and each thread then stores kDecodeWaves
// consecutive words (64 bytes) of one transposed row.
__device__ __forceinline__ bool line_interval(const LineOp &op, int W, int &s, int &e)
{
    const int right = op.w - 1 - op.c;
    if (op.mode == kLineErode || op.mode == kLineOpen) {
        const int ns = (s == 0) ? 0 : s + op.c;
        const int ne = (e == W) ? W : e - right;
        if (ns >= ne) return false;
        s = ns;
        e = ne;
    }
    if (op.mode == kLineDilate || op.mode == kLineOpen) {
        s = max(0, s - op.c);
        e = min(W, e + right);
    }
    return s < e;
}

constexpr int kDecodeWaves = 8;         // row blocks per workgroup = words per stored segment
constexpr int kDecodeStrip = 8;         // words of a row one workgroup decodes
constexpr int kDecodePad = kDecodeWaves + 1;

__global__ __launch_bounds__(64 * kDecodeWaves) void decode_transpose_kernel(
    const int *__restrict__ row_ptr, const int *__restrict__ runs, long long cap, int W, int H,
    int nw, int nk, int nstrips, int kgroups, long long total, uint64_t *__restrict__ dst, int dstride,
    long long dpw, LineOp op, unsigned long long *trace)
{
    __shared__ uint64_t stage[kDecodeStrip * 64 * kDecodePad];
    const long long g = xcd_block();
    if (g >= total) return;                 // whole workgroup
    const int lane = lane_id(), q = (int)(threadIdx.x >> 6);
    const long long per_page = (long long)nstrips * kgroups;
    const int page = (int)(g / per_page);
    const int u = (int)(g - (long long)page * per_page);
    const int strip = u / kgroups, kg = u - strip * kgroups;
    const int k0 = kg * kDecodeWaves, k = k0 + q;
    const int j0 = strip * kDecodeStrip, j1 = min(j0 + kDecodeStrip, nw);
    const int y = 64 * k + lane;
    const bool live = y < H;
    const int reach = op.w - 1;
    const int2 *rr = reinterpret_cast<const int2 *>(runs);
    int n = 0, ni = 0, i = 0, prev_e = 0;   // next interval to load; gaps: end of the run before it
    if (live) {
        const long long r = (long long)page * H + y;
        const long long b0 = min((long long)max(row_ptr[r], 0), cap);
        const long long b1 = max(b0, min((long long)row_ptr[r + 1], cap));
        n = (int)(b1 - b0);
        rr += b0;
        ni = op.comp ? n + 1 : n;           // intervals: runs, or the n + 1 gaps
        if (trace && strip == 0) trace_add(trace, (unsigned long long)n, 0);
        // first interval whose raw end + reach passes the strip's first pixel
        const int x0 = 64 * j0;
        int hi = ni;
        while (i < hi) {
            const int mid = (i + hi) >> 1;
            const int e = op.comp ? (mid == n ? W : rr[mid].x) : rr[mid].y;
            if (e + reach > x0) hi = mid; else i = mid + 1;
        }
        if (op.comp && i > 0) prev_e = rr[i - 1].y;
    }
    bool have = false;                      // (a, b): the interval carried into the next word
    int a = 0, b = 0;
    for (int j = j0; j < j1; j++) {
        uint64_t v = 0;
        if (live) {
            const int x0 = 64 * j, x1 = min(x0 + 64, W);
            for (;;) {
                if (!have) {
                    if (i >= ni) break;
                    int s, e;
                    if (op.comp) {
                        s = prev_e;
                        if (i < n) {
                            const int2 t = rr[i];
                            e = t.x;
                            prev_e = t.y;
                        } else {
                            e = W;
                        }
                    } else {
                        const int2 t = rr[i];
                        s = t.x;
                        e = t.y;
                    }
                    i++;
                    if (!line_interval(op, W, s, e)) continue;
                    a = s;
                    b = e;
                    have = true;
                }
                if (a >= x1) break;         // starts in a later word
                const int lo = max(a, x0) - x0, hi = min(b, x1) - x0;
                if (lo < hi) v |= (~0ull >> (64 - (hi - lo))) << lo;   // bits lo .. hi - 1
                if (b > x1) break;          // reaches into the next word
                have = false;
            }
            if (op.comp) {
                const int nb = x1 - x0;
                v = ~v & ((nb == 64) ? ~0ull : ((1ull << nb) - 1));
            }
        }
        v = wave_transpose64(v);            // lane: transposed row 64j + lane, word k
        stage[((j - j0) * 64 + lane) * kDecodePad + q] = v;
    }
    __syncthreads();
    // thread t: transposed row 64(j0 + t / 64) + t % 64, words k0 .. k0 + kDecodeWaves - 1
    const int jj = (int)(threadIdx.x >> 6);
    const int x = 64 * (j0 + jj) + lane;
    const int nkk = min(kDecodeWaves, nk - k0);
    if (j0 + jj < j1 && x < W) {
        const uint64_t *sv = stage + (jj * 64 + lane) * kDecodePad;
        uint64_t *dp = dst + (long long)page * dpw + (long long)x * dstride + k0;
        if (nkk == kDecodeWaves && (((uintptr_t)dp) & 15) == 0) {
            ulonglong2 *d2 = reinterpret_cast<ulonglong2 *>(dp);
#pragma unroll
            for (int c = 0; c < kDecodeWaves / 2; c++) d2[c] = make_ulonglong2(sv[2 * c], sv[2 * c + 1]);
        } else {
            for (int c = 0; c < nkk; c++) dp[c] = sv[c];
        }
    }
}

// ------------------------------------------------- rows in two layouts
// Between passes the library keeps run-length rows in a slot layout: row r
// owns runs r*cap .. r*cap+cap-1 and cnt[r] of them are used, cap being the
// most runs a row of the image width can have.  A pass can then write its
// rows without knowing where earlier rows end, so no scan is needed until
// the final result is packed into CSR form.
struct RowsIn {
    const int *rp;          // CSR offsets, or nullptr for the slot layout
    const int *cnt;         // slot layout: runs per row
    const int *runs;
    long long cap;          // CSR: runs the array holds; slot: runs per row
};

__device__ __forceinline__ void row_span(const RowsIn &v, long long r, long long &base, int &n)
{
    if (v.rp) {
        base = min((long long)max(v.rp[r], 0), v.cap);
        n = (int)max(0LL, min((long long)v.rp[r + 1], v.cap) - base);
    } else {
        base = r * v.cap;
        n = min(max(v.cnt[r], 0), (int)v.cap);
    }
}

constexpr int kGroup = 16;                        // lanes that share one row
constexpr int kGroupsPerBlock = 256 / kGroup;
// Rows of up to kStageRuns runs are loaded whole before they are used: into
// registers (kARegs runs per lane) or a per-group LDS window.
constexpr int kStageRuns = 128;
constexpr int kARegs = kStageRuns / kGroup;

__device__ __forceinline__ int glane() { return (int)(threadIdx.x & (kGroup - 1)); }

// This group's 16 bits of a wave-wide ballot.
__device__ __forceinline__ unsigned group_ballot(bool p)
{
    const unsigned long long m = __ballot(p);
    return (unsigned)(m >> (lane_id() & ~(kGroup - 1))) & 0xffffu;
}

// Inclusive prefix sum over the 16 lanes of a group.  A DPP row is 16
// lanes, so row_shr moves values within the group only and lanes below the
// shift read 0: no LDS traffic.
__device__ __forceinline__ int group_incl_scan(int x)
{
    x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, false);    // row_shr:1
    x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, false);    // row_shr:2
    x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, false);    // row_shr:4
    x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, false);    // row_shr:8
    return x;
}

// Lane 0 of this lane's group (DPP row_newbcast:0).
__device__ __forceinline__ int group_first(int x)
{
    return __builtin_amdgcn_update_dpp(0, x, 0x150, 0xf, 0xf, false);
}

// Lane 15 of this lane's group (DPP row_newbcast:15).
__device__ __forceinline__ int group_last(int x)
{
    return __builtin_amdgcn_update_dpp(0, x, 0x15f, 0xf, 0xf, false);
}

// Inclusive maximum over the 16 lanes of a group (lanes below the shift
// read -1, the "none" value of the callers).
__device__ __forceinline__ int group_incl_max(int x)
{
    x = max(x, __builtin_amdgcn_update_dpp(-1, x, 0x111, 0xf, 0xf, false));    // row_shr:1
    x = max(x, __builtin_amdgcn_update_dpp(-1, x, 0x112, 0xf, 0xf, false));    // row_shr:2
    x = max(x, __builtin_amdgcn_update_dpp(-1, x, 0x114, 0xf, 0xf, false));    // row_shr:4
    x = max(x, __builtin_amdgcn_update_dpp(-1, x, 0x118, 0xf, 0xf, false));    // row_shr:8
    return x;
}

// ------------------------------------------- packed -> runs, narrow rows
// The same transitions with one 16-lane group per row (four rows a wave):
// lane k takes words k, k + 16, ...; the bit before a word comes from the
// lane before (DPP row_shr) or, for lane 0, from lane 15 of the block
// before.  A row of 40 words is three blocks instead of a wave with 24 idle
// lanes, and a quarter of the waves.  Used for rows of up to 128 words.
constexpr int kNarrowRowWords = 128;

template <bool EMIT>
__global__ __launch_bounds__(256) void pack_to_rle_group_kernel(
    const uint64_t *__restrict__ words, int nw, int stride, int H, int R, long long page_words,
    uint64_t padmask, int *__restrict__ counts, const int *__restrict__ row_ptr,
    int *__restrict__ runs, long long cap, unsigned long long *trace)
{
    const int r = (int)(blockIdx.x * (unsigned)kGroupsPerBlock + (threadIdx.x >> 4));
    if (r >= R) return;                    // whole group
    const int gl = glane();
    const int page = r / H, y = r - page * H;
    const uint64_t *row = words + (long long)page * page_words + (long long)y * stride;
    const long long obase = EMIT ? row_ptr[r] : 0;
    const int capi = (int)min(cap, 0x7fffffffLL);   // run indices fit in int: row offsets are int
    int cstart = 0, cend = 0;
    int prev = 0;                          // bit 63 of the word before this block
    int last_start = -1;                   // the last start before this block (-1: none)
    // the whole row first (every load in flight at once), then its blocks
    constexpr int kBlk = kNarrowRowWords / kGroup + 1;
    uint64_t wv[kBlk];
#pragma unroll
    for (int m = 0; m < kBlk; m++) {
        const int j = m * kGroup + gl;
        wv[m] = j < nw ? row[j] : 0ull;
        if (j == nw - 1) wv[m] &= padmask;
    }
#pragma unroll
    for (int m = 0; m < kBlk; m++) {
        const int j0 = m * kGroup;
        if (j0 > nw) break;                // wave-uniform
        const int j = j0 + gl;
        const uint64_t a = wv[m];
        const int top = (int)(a >> 63);
        const int up = __builtin_amdgcn_update_dpp(prev, top, 0x111, 0xf, 0xf, false);   // row_shr:1
        const uint64_t sh = (a << 1) | (uint64_t)(unsigned)up;
        uint64_t st = a & ~sh, en = ~a & sh;
        if (j > nw) {
            st = 0;
            en = 0;
        }
        // blocks without a transition in all four rows of the wave (the
        // white space between text lines) change no row's state
        if (__builtin_amdgcn_ballot_w64((st | en) != 0) == 0) continue;
        // a row has as many ends as starts: the count pass scans the starts,
        // the emit pass only the ends
        const int ns = EMIT ? 0 : __popcll(st), ne = EMIT ? __popcll(en) : 0;
        const int is = EMIT ? 0 : group_incl_scan(ns), ie = EMIT ? group_incl_scan(ne) : 0;
        if (EMIT) {
            // every run is written whole, as one pair, by the lane that holds
            // its end: its start is the nearest start bit below the end in
            // the same word, or else the last start of an earlier word (runs
            // alternate with gaps, so that is the run's own start)
            const int ls = st ? 64 * j + 63 - (int)__clzll(st) : -1;
            const int incl = group_incl_max(ls);
            const int before = max(last_start, __builtin_amdgcn_update_dpp(-1, incl, 0x111, 0xf, 0xf, false));
            emit_word_runs(st, en, 64 * j, before, (int)(obase + cend + ie - ne), capi, runs);
            last_start = max(last_start, group_last(incl));
        }
        if (EMIT) cend += group_last(ie); else cstart += group_last(is);
        prev = group_last(top);
    }
    if (!EMIT && gl == 0) counts[r] = cstart;
    if (EMIT && trace && gl == 0) trace_add(trace, 0, (unsigned long long)cend);
}

// ---------------------------------------- packed -> runs of the transpose
// The run counts of the transposed rows come with the transpose, one per
// piece of a row (the part a transpose tile covers); this sums each row's
// pieces.
__global__ __launch_bounds__(256) void piece_sum_kernel(const int *__restrict__ pieces, int per_row, long long R,
                                                        int *__restrict__ counts)
{
    const long long r = (long long)blockIdx.x * 256 + threadIdx.x;
    if (r >= R) return;
    int s = 0;
    for (int k = 0; k < per_row; k++) s += pieces[k * R + r];    // piece-major
    counts[r] = s;
}

// The number of 16-run blocks the longest of the wave's four rows needs
// (n <= kStageRuns runs each), read from one lane of each group: loops over
// register blocks end on a uniform branch.  Groups that left early leave
// stale values in their lanes: compared unsigned and clamped, they can only
// raise the bound, to at most the blocks of kStageRuns runs.
__device__ __forceinline__ int wave_blocks(int n)
{
    const unsigned m = max(max((unsigned)__builtin_amdgcn_readlane(n, 0), (unsigned)__builtin_amdgcn_readlane(n, 16)),
                           max((unsigned)__builtin_amdgcn_readlane(n, 32), (unsigned)__builtin_amdgcn_readlane(n, 48)));
    return (int)((min(m, (unsigned)kStageRuns) + kGroup - 1) / kGroup);
}

// ------------------------------------------------------ within-line pass
// Erosion of every row by a 1 x w element with origin cx (section "Within-
// Line Morphological Operations"): run [s, e) becomes [s + cx, e - (w-1-cx)),
// a side lying on the row border stays put (outside pixels are 1), and runs
// that vanish are dropped.  With comp_in the rows' complements are eroded:
// the gaps between runs, including the ones at both ends, play the runs.
// One group of 16 lanes per row, lanes over runs, compaction by ballot.
// With keep_whole the candidates that survive the erosion are written as
// they were: the opening by a one-row element (section "Within-Line
// Morphological Operations": a run survives erosion and dilation unchanged
// when it is at least as long as the element, the border runs by their
// shrunk length), and on the gaps, the closing's complement.
__global__ __launch_bounds__(256) void row_erode_kernel(RowsIn in, int R, int W, int w, int cx, int comp_in,
                                                        int keep_whole, int *__restrict__ out_cnt,
                                                        int *__restrict__ out_runs, long long cap_row,
                                                        unsigned long long *trace)
{
    const long long r = (long long)xcd_block() * kGroupsPerBlock + (threadIdx.x >> 4);
    if (r >= R) return;                    // whole group
    const int gl = glane();
    long long base;
    int n;
    row_span(in, r, base, n);
    const int *rr = in.runs + 2 * base;
    const int ncand = comp_in ? n + 1 : n;
    const int right = w - 1 - cx;
    int *o = out_runs + 2 * r * cap_row;
    int carry = 0;
    // candidate k -> kept run (ns, ne) at the next free slot
    auto emit = [&](int k, int s, int e) {
        const int ns = (s == 0) ? 0 : s + cx;
        const int ne = (e == W) ? W : e - right;
        const bool keep = k < ncand && s < e && ns < ne;
        const unsigned gm = group_ballot(keep);
        const int idx = carry + __popc(gm & ((1u << gl) - 1));
        if (keep && idx < cap_row) ((int2 *)o)[idx] = keep_whole ? make_int2(s, e) : make_int2(ns, ne);
        carry += __popc(gm);
    };
    if (ncand <= kStageRuns) {
        // the whole row in registers (lane k holds runs k + 16 m), every load
        // issued before the first use
        const int2 *r2 = (const int2 *)rr;
        const int nblk = wave_blocks(ncand);
        int2 v[kARegs];
#pragma unroll
        for (int m = 0; m < kARegs; m++) {
            if (m >= nblk) break;
            const int k = m * kGroup + gl;
            v[m] = k < n ? r2[k] : make_int2(0, 0);
        }
        int prev_end = 0;                   // end of run 16 m - 1
#pragma unroll
        for (int m = 0; m < kARegs; m++) {
            if (m * kGroup >= ncand) break;
            const int k = m * kGroup + gl;
            int s, e;
            if (comp_in) {
                // gap k lies between the end of run k - 1 (the lane before,
                // or lane 15 of the previous block) and the start of run k
                const int pe = __builtin_amdgcn_update_dpp(prev_end, v[m].y, 0x111, 0xf, 0xf, false);
                s = (k == 0) ? 0 : pe;
                e = (k == n) ? W : v[m].x;
                prev_end = group_last(v[m].y);
            } else {
                s = v[m].x;
                e = v[m].y;
            }
            emit(k, s, e);
        }
    } else {
        for (int k0 = 0; k0 < ncand; k0 += kGroup) {
            const int k = k0 + gl;
            int s = 0, e = 0;
            if (k < ncand) {
                if (comp_in) {
                    s = (k == 0) ? 0 : rr[2 * k - 1];
                    e = (k == n) ? W : rr[2 * k];
                } else {
                    s = rr[2 * k];
                    e = rr[2 * k + 1];
                }
            }
            emit(k, s, e);
        }
    }
    if (gl == 0) {
        out_cnt[r] = (int)min((long long)carry, cap_row);
        if (trace) trace_add(trace, (unsigned long long)n, (unsigned long long)carry);
    }
}

// ----------------------------------------------------- between-line pass
// The first doubling step of a chain reads its rows straight from the input
// and applies the within-line erosion as it reads them (there is no
// separate within-line launch then).  Candidate k of a row is its run k, or
// with comp the gap before run k (gap n runs to the right border), shrunk by
// cx on the left and `right` on the right unless that side lies on a border.
// A candidate that vanishes keeps s >= e and is skipped; starts and ends
// still ascend with k, so the searches below need no compaction.
struct RowX {
    int cx, right, comp, W;
};

__device__ __forceinline__ int2 shrink(const RowX &x, int s, int e)
{
    return make_int2(s == 0 ? 0 : s + x.cx, e == x.W ? x.W : e - x.right);
}

__device__ __forceinline__ bool live(int2 c) { return c.x < c.y; }

// Candidate k of a stored row R of n runs (k < n, or k <= n with comp).
template <bool ROWX>
__device__ __forceinline__ int2 cand(const RowX &x, const int *R, int n, int k)
{
    if (!ROWX) return make_int2(R[2 * k], R[2 * k + 1]);
    if (x.comp) return shrink(x, k == 0 ? 0 : R[2 * k - 1], k == n ? x.W : R[2 * k]);
    return shrink(x, R[2 * k], R[2 * k + 1]);
}

// Whether a row's live candidates cover pixel 0 and pixel W-1.  Only the
// first candidate can start at 0 and only the last can end at W.
template <bool ROWX>
__device__ __forceinline__ void row_ends(const RowX &x, const int *R, int n, int W, bool &has0, bool &hasW)
{
    const int nc = n + ((ROWX && x.comp) ? 1 : 0);
    if (nc == 0) {
        has0 = hasW = false;
        return;
    }
    const int2 f = cand<ROWX>(x, R, n, 0), l = cand<ROWX>(x, R, n, nc - 1);
    has0 = live(f) && f.x == 0;
    hasW = live(l) && l.y == W;
}

// Intersection of the rows A (na candidates) and B (nb candidates) into o,
// by the lanes of one group: lane k takes candidates k, k+16, ... of A,
// finds the first candidate of B that ends after it starts, and emits every
// overlap with a live candidate in order.
template <bool ROWX>
__device__ __forceinline__ int group_intersect(const RowX &x, const int *A, int na_raw, int na, const int *B,
                                               int nb_raw, int nb, int *o, long long cap_row)
{
    const int gl = glane();
    int carry = 0;
    for (int k0 = 0; k0 < na; k0 += kGroup) {
        const int k = k0 + gl;
        int c = 0, span = 0, j0 = 0, sa = 0, ea = 0;
        if (k < na) {
            const int2 ca = cand<ROWX>(x, A, na_raw, k);
            sa = ca.x;
            ea = ca.y;
        }
        if (k < na && sa < ea) {
            int lo = 0, hi = nb;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (cand<ROWX>(x, B, nb_raw, mid).y > sa) hi = mid; else lo = mid + 1;
            }
            j0 = lo;
            for (int j = j0; j < nb; j++) {
                const int2 cb = cand<ROWX>(x, B, nb_raw, j);
                if (cb.x >= ea) break;
                span++;
                c += live(cb);
            }
        }
        const int inc = group_incl_scan(c);
        long long idx = carry + inc - c;
        for (int j = j0; j < j0 + span; j++) {
            const int2 cb = cand<ROWX>(x, B, nb_raw, j);
            if (!live(cb)) continue;
            if (idx < cap_row) {
                o[2 * idx] = max(sa, cb.x);
                o[2 * idx + 1] = min(ea, cb.y);
            }
            idx++;
        }
        carry += group_last(inc);
    }
    return carry;
}

// The same intersection with row A in registers (lane k holds runs k + 16 m
// of A) and row B staged in this group's LDS window.  Every load of both
// rows has been issued before the first search step, so a group waits for
// global memory twice (counts, then runs) instead of once per search step.

__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
}

template <bool ROWX>
__device__ __forceinline__ int group_intersect_staged(const int2 (&a)[kARegs], int na, const int2 *sB, int nb,
                                                      int2 *__restrict__ o, int cap)
{
    const int gl = glane();
    int carry = 0;
#pragma unroll
    for (int m = 0; m < kARegs; m++) {
        if (m * kGroup >= na) break;
        const int k = m * kGroup + gl;
        const int sa = a[m].x, ea = a[m].y;
        int c = 0, span = 0, j0 = 0;
        int2 b0 = make_int2(0, 0), b1 = make_int2(0, 0);
        bool e0 = false, e1 = false;        // b0, b1 overlap and are emitted
        if (k < na && sa < ea) {
            // j0 = the first candidate of B that ends after sa (ends ascend)
            int lo = 0, hi = nb;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (sB[mid].y > sa) hi = mid; else lo = mid + 1;
            }
            j0 = lo;
            // most runs overlap at most two runs of the other row: those two
            // stay in registers for the emission
            b0 = sB[min(j0, nb - 1)];
            b1 = sB[min(j0 + 1, nb - 1)];
            const bool h0 = j0 < nb && b0.x < ea;
            const bool h1 = h0 && j0 + 1 < nb && b1.x < ea;
            e0 = h0 && (!ROWX || live(b0));
            e1 = h1 && (!ROWX || live(b1));
            span = (int)h0 + (int)h1;
            c = (int)e0 + (int)e1;
            if (h1) {
#pragma unroll 1
                for (int j = j0 + 2; j < nb && sB[j].x < ea; j++) {
                    span++;
                    c += ROWX ? (int)live(sB[j]) : 1;
                }
            }
        }
        const int inc = group_incl_scan(c);
        int idx = carry + inc - c;
        if (e0) {
            if (idx < cap) o[idx] = make_int2(max(sa, b0.x), min(ea, b0.y));
            idx++;
        }
        if (e1) {
            if (idx < cap) o[idx] = make_int2(max(sa, b1.x), min(ea, b1.y));
            idx++;
        }
#pragma unroll 1
        for (int q = 2; q < span; q++) {
            const int2 b = sB[j0 + q];
            if (ROWX && !live(b)) continue;
            if (idx < cap) o[idx] = make_int2(max(sa, b.x), min(ea, b.y));
            idx++;
        }
        carry += group_last(inc);
    }
    return carry;
}

// Candidates of a row held in registers (lane k holds raw runs k + 16 m):
// in place, the gaps of the complement taking the end of the run before
// from the lane before (or lane 15 of the block before).
__device__ __forceinline__ void shrink_regs(const RowX &x, int2 (&v)[kARegs], int n, int nblk)
{
    const int gl = glane();
    int prev_end = 0;
#pragma unroll
    for (int m = 0; m < kARegs; m++) {
        if (m >= nblk) break;                  // wave-uniform
        const int k = m * kGroup + gl;
        if (x.comp) {
            const int pe = __builtin_amdgcn_update_dpp(prev_end, v[m].y, 0x111, 0xf, 0xf, false);
            const int lastend = group_last(v[m].y);
            v[m] = shrink(x, k == 0 ? 0 : pe, k == n ? x.W : v[m].x);
            prev_end = lastend;
        } else {
            v[m] = shrink(x, v[m].x, v[m].y);
        }
    }
}

// One doubling step between lines (sections "Between Line Boolean
// Operations" and "Efficient Binary Decompositions"): output row r of a page
// is the intersection of rows r and r + K of the input, where input row x is
// stored row x - off if that lies in [0, real), and otherwise a full row
// [0, W) (outside the image erosion sees 1s).  NA rows per page come in,
// NA - K go out.  One group of lanes per output row.
// n / d for 0 <= n < 2^31 as a multiply-high, an add and a shift, with
// the round-up multiplier m = floor(2^32 (2^l - d) / d) + 1, l = ceil(log2 d)
// (Granlund and Montgomery, "Division by invariant integers using
// multiplication"): the wave-uniform divisor's quotient costs three VALU
// instructions instead of a reciprocal sequence.
struct DivU {
    unsigned mul;
    int shift;
};

static DivU div_by(unsigned d)
{
    int l = 0;
    while ((1ull << l) < d) l++;
    const unsigned long long m = ((1ull << 32) * ((1ull << l) - d)) / d + 1;
    return DivU{(unsigned)m, l};
}

__device__ __forceinline__ unsigned div_u(unsigned n, DivU q) { return (__umulhi(n, q.mul) + n) >> q.shift; }

template <bool ROWX>
__global__ __launch_bounds__(256) void col_and_kernel(RowsIn in, int off, int real, int NA, int K, DivU nbd, int P,
                                                      int W, RowX x, int *__restrict__ out_cnt,
                                                      int *__restrict__ out_runs, long long cap_row,
                                                      int *__restrict__ gap_cnt, unsigned long long *trace)
{
    // gap_cnt (the last step of a chain whose result is complemented): also
    // the run count of each output row's complement, which is its run count
    // plus one, less one for each border pixel the row covers
    __shared__ int2 stage[kGroupsPerBlock][kStageRuns];
    const int NB = NA - K;
    const long long t = (long long)xcd_block() * kGroupsPerBlock + (threadIdx.x >> 4);
    if (t >= (long long)P * NB) return;     // whole group
    const int gl = glane();
    // the host keeps every row index below 2^31: 32-bit division
    const unsigned tu = (unsigned)t;
    const int page = (int)div_u(tu, nbd), r = (int)(tu - (unsigned)page * (unsigned)NB);
    const int ia = r - off, ib = r + K - off;
    const bool va = ia >= 0 && ia < real, vb = ib >= 0 && ib < real;
    int *o = out_runs + 2 * t * cap_row;
    if (!va && !vb) {
        if (gl == 0) {
            o[0] = 0;
            o[1] = W;
            out_cnt[t] = 1;
            if (gap_cnt) gap_cnt[t] = 0;
            if (trace) trace_add(trace, 0, 1ull);
        }
        return;
    }
    const int extra = (ROWX && x.comp) ? 1 : 0;      // a row of n runs has n + extra candidates
    if (!va || !vb) {                       // full row AND x = x
        long long base;
        int n;
        row_span(in, (long long)page * real + (va ? ia : ib), base, n);
        const int *src = in.runs + 2 * base;
        int cnt = 0;
        if (!ROWX) {
            n = (int)min((long long)n, cap_row);
            for (int k = gl; k < n; k += kGroup) {
                o[2 * k] = src[2 * k];
                o[2 * k + 1] = src[2 * k + 1];
            }
            cnt = n;
        } else {
            // the live candidates, compacted by ballot
            const int nc = n + extra;
            for (int k0 = 0; k0 < nc; k0 += kGroup) {
                const int k = k0 + gl;
                const int2 c = k < nc ? cand<true>(x, src, n, k) : make_int2(0, 0);
                const bool keep = k < nc && live(c);
                const unsigned gm = group_ballot(keep);
                const int idx = cnt + __popc(gm & ((1u << gl) - 1));
                if (keep && idx < cap_row) ((int2 *)o)[idx] = c;
                cnt += __popc(gm);
            }
            cnt = (int)min((long long)cnt, cap_row);
        }
        if (gl == 0) {
            out_cnt[t] = cnt;
            if (gap_cnt) {
                bool h0, hW;
                row_ends<ROWX>(x, src, n, W, h0, hW);
                gap_cnt[t] = cnt + 1 - (int)h0 - (int)hW;
            }
            // input runs: the A row (if stored); the B row only where it is
            // never an A row (r + K >= NB)
            if (trace)
                trace_add(trace, (unsigned long long)((va ? n : 0) + (vb && r + K >= NB ? n : 0)),
                          (unsigned long long)cnt);
        }
        return;
    }
    long long ba, bb;
    int na, nb;
    row_span(in, (long long)page * real + ia, ba, na);
    row_span(in, (long long)page * real + ib, bb, nb);
    const int *A = in.runs + 2 * ba;
    const int *B = in.runs + 2 * bb;
    // the intersection is symmetric: the shorter row goes to registers and
    // its candidates to the lanes, the longer one is searched
    const bool swap = nb < na;
    const int *S = swap ? B : A, *L = swap ? A : B;
    const int ns = min(na, nb), nl = max(na, nb);        // runs stored
    const int cs = ns + extra, cl = nl + extra;           // candidates
    int cnt = 0;
    if (cs == 0) {
        cnt = 0;
    } else if (cl <= kStageRuns) {
        // the blocks of 16 candidates that any row pair of this wave needs
        const int nblk = wave_blocks(cl);
        const int2 *S2 = (const int2 *)S, *L2 = (const int2 *)L;
        int2 a[kARegs], b[kARegs];
#pragma unroll
        for (int m = 0; m < kARegs; m++) {
            if (m >= nblk) break;
            const int k = m * kGroup + gl;
            a[m] = k < ns ? S2[k] : make_int2(0, 0);
            b[m] = k < nl ? L2[k] : make_int2(0, 0);
        }
        if (ROWX) {
            shrink_regs(x, a, ns, nblk);
            shrink_regs(x, b, nl, nblk);
        }
        int2 *sB = stage[threadIdx.x >> 4];
#pragma unroll
        for (int m = 0; m < kARegs; m++) {
            if (m >= nblk) break;
            if (m * kGroup + gl < cl) sB[m * kGroup + gl] = b[m];
        }
        wave_lds_sync();
        cnt = group_intersect_staged<ROWX>(a, cs, sB, cl, (int2 *)o, (int)cap_row);
    } else {
        cnt = group_intersect<ROWX>(x, S, ns, cs, L, nl, cl, o, cap_row);
    }
    if (gl == 0) {
        out_cnt[t] = (int)min((long long)cnt, cap_row);
        if (gap_cnt) {
            bool a0, aW, b0, bW;
            row_ends<ROWX>(x, A, na, W, a0, aW);
            row_ends<ROWX>(x, B, nb, W, b0, bW);
            gap_cnt[t] = (int)min((long long)cnt, cap_row) + 1 - (int)(a0 && b0) - (int)(aW && bW);
        }
        if (trace) trace_add(trace, (unsigned long long)(na + (r + K >= NB ? nb : 0)), (unsigned long long)cnt);
    }
}

// ------------------------------------------- runs -> packed, narrow rows
// One 16-lane group per row of up to 128 words (four rows a wave): the row
// is cleared in this group's LDS buffer, each lane ORs its intervals in
// (the words an interval covers whole are stored, the partial words at its
// ends ORed), and the row goes out in 128-byte pieces.  With a within-line
// operation (op.mode != kLineNone) each run, or with op.comp each gap
// between runs (including the two at the borders), is first eroded,
// dilated or opened along the row, and with op.comp the row is then
// complemented.  Dilated intervals may overlap; every write is an OR or a
// store of all ones, so the order does not matter.  Interval bounds are
// clamped to the row and offsets to the run capacity, so damaged input
// cannot reach outside either buffer.
__global__ __launch_bounds__(256) void rle_to_pack_group_kernel(const int *__restrict__ row_ptr,
                                                                const int *__restrict__ runs, int nw,
                                                                int R, int H, int W, uint64_t *__restrict__ words,
                                                                int stride, long long page_words, long long cap,
                                                                LineOp op, unsigned long long *trace)
{
    __shared__ uint64_t rowbuf[kGroupsPerBlock][kNarrowRowWords];
    const int r = (int)(blockIdx.x * (unsigned)kGroupsPerBlock + (threadIdx.x >> 4));
    if (r >= R) return;                    // whole group; only wave-level syncs below
    const int gl = glane();
    uint64_t *buf = rowbuf[threadIdx.x >> 4];
    for (int j = gl; j < nw; j += kGroup) buf[j] = 0;
    wave_lds_sync();
    const long long b0 = min((long long)max(row_ptr[r], 0), cap);
    const long long b1 = max(b0, min((long long)row_ptr[r + 1], cap));
    const int n = (int)(b1 - b0);
    const int2 *rr = reinterpret_cast<const int2 *>(runs) + b0;
    const int xmax = 64 * nw;
    const int ni = op.comp ? n + 1 : n;
    for (int k = gl; k < ni; k += kGroup) {
        int s0, e0;
        if (op.comp) {
            s0 = (k == 0) ? 0 : rr[k - 1].y;
            e0 = (k == n) ? W : rr[k].x;
        } else {
            const int2 v = rr[k];
            s0 = v.x;
            e0 = v.y;
        }
        if (op.mode != kLineNone && !line_interval(op, W, s0, e0)) continue;
        s0 = max(s0, 0);
        e0 = min(e0, xmax);
        if (s0 >= e0) continue;
        const int ws = s0 >> 6, we = (e0 - 1) >> 6;
        const uint64_t lo = ~0ull << (s0 & 63);
        const uint64_t hi = ~0ull >> (63 - ((e0 - 1) & 63));
        if (ws == we) {
            atomicOr((unsigned long long *)&buf[ws], (unsigned long long)(lo & hi));
        } else {
            atomicOr((unsigned long long *)&buf[ws], (unsigned long long)lo);
            for (int w = ws + 1; w < we; w++) buf[w] = ~0ull;
            atomicOr((unsigned long long *)&buf[we], (unsigned long long)hi);
        }
    }
    wave_lds_sync();
    const int page = r / H, y = r - page * H;
    uint64_t *out = words + (long long)page * page_words + (long long)y * stride;
    for (int j = gl; j < nw; j += kGroup) {
        uint64_t v = buf[j];
        if (op.comp) {
            const int nb = min(64, W - 64 * j);
            v = ~v & ((nb >= 64) ? ~0ull : ((1ull << nb) - 1));
        }
        out[j] = v;
    }
    if (trace && gl == 0) trace_add(trace, (unsigned long long)n, 0);
}

// ----------------------------------------------------- block prefix scans
// Between-line erosion by h rows in two launches for tall elements: the
// extended rows 0 .. NA-1 of a page (row x = stored row x - off, a full
// row outside) fall into blocks of h rows; one group per block walks it
// down, writing G(x) = E(x0) AND ... AND E(x), and one walks it up,
// writing F(x) = E(x) AND ... AND E(x1 - 1), E being the row after the
// within-line pass (ROWX).  Output row y is then F(y) AND G(y + h - 1):
// the two ranges meet to cover y .. y + h - 1 (when y starts a block,
// G(y + h - 1) is the whole block, which F(y) already is).  F(x) is
// stored at row x and G(x) at row NA + x of a page of 2 NA slot rows, so
// the combining step is col_and_kernel<false> with K = NA + h - 1.
// The current row of a walk stays in the group's LDS window (global
// memory, behind a fence, when it has more than kScanWin runs).
constexpr int kScanWin = 64;             // runs of the current row a group keeps in LDS (16 KiB a workgroup)

template <bool ROWX>
__global__ __launch_bounds__(256) void col_scan_kernel(RowsIn in, int off, int real, int NA, int h, int nblk, int P,
                                                       int W, RowX x, int *__restrict__ out_cnt,
                                                       int *__restrict__ out_runs, long long cap_row,
                                                       unsigned long long *trace)
{
    __shared__ int2 win[kGroupsPerBlock][2][kScanWin];
    const long long t = (long long)xcd_block() * kGroupsPerBlock + (threadIdx.x >> 4);
    if (t >= (long long)P * nblk * 2) return;        // whole group
    const int gl = glane();
    const int dir = (int)(t & 1);                    // 0: down (G), 1: up (F)
    const long long pb = t >> 1;
    const int page = (int)(pb / nblk), blk = (int)(pb - (long long)page * nblk);
    const int x0 = blk * h, x1 = min(x0 + h, NA);
    const int extra = (ROWX && x.comp) ? 1 : 0;
    int2 *wa = win[threadIdx.x >> 4][0], *wb = win[threadIdx.x >> 4][1];
    const int2 *cur = wa;                            // the current row: LDS window or a stored output row
    int ncur = 0;
    unsigned long long rin = 0, rout = 0;
    for (int s = 0; s < x1 - x0; s++) {
        const int xr = dir == 0 ? x0 + s : x1 - 1 - s;
        const long long orow = (long long)page * 2 * NA + (dir == 0 ? NA + xr : xr);
        int2 *o = reinterpret_cast<int2 *>(out_runs) + orow * cap_row;
        const int ir = xr - off;
        const bool stored = ir >= 0 && ir < real;
        long long base = 0;
        int n = 0;
        if (stored) row_span(in, (long long)page * real + ir, base, n);
        const int *R = in.runs + 2 * base;
        if (dir == 0) rin += n;
        int cnt = 0;
        if (s == 0 || (s > 0 && ncur > 0 && !stored)) {
            // the row itself (first step), or the current row unchanged (a full row meets it)
            if (s == 0 && !stored) {
                if (gl == 0) {
                    o[0] = make_int2(0, W);
                    wb[0] = make_int2(0, W);
                }
                cnt = 1;
            } else if (s == 0) {
                const int nc = n + extra;
                for (int k0 = 0; k0 < nc; k0 += kGroup) {
                    const int k = k0 + gl;
                    const int2 c = k < nc ? cand<ROWX>(x, R, n, k) : make_int2(0, 0);
                    const bool keep = k < nc && live(c);
                    const unsigned gm = group_ballot(keep);
                    const int idx = cnt + __popc(gm & ((1u << gl) - 1));
                    if (keep && idx < cap_row) {
                        o[idx] = c;
                        if (idx < kScanWin) wb[idx] = c;
                    }
                    cnt += __popc(gm);
                }
            } else {
                for (int k = gl; k < ncur; k += kGroup) {
                    const int2 c = cur[k];
                    o[k] = c;
                    if (k < kScanWin) wb[k] = c;
                }
                cnt = ncur;
            }
        } else if (ncur > 0) {
            // cur AND the candidates of the row: lanes over the row's candidates
            const int nc = n + extra;
            int carry = 0;
            for (int k0 = 0; k0 < nc; k0 += kGroup) {
                const int k = k0 + gl;
                int c = 0, span = 0, j0 = 0, sa = 0, ea = 0;
                if (k < nc) {
                    const int2 a = cand<ROWX>(x, R, n, k);
                    sa = a.x;
                    ea = a.y;
                }
                if (k < nc && sa < ea) {
                    int lo = 0, hi = ncur;           // the first run of cur that ends after sa
                    while (lo < hi) {
                        const int mid = (lo + hi) >> 1;
                        if (cur[mid].y > sa) hi = mid; else lo = mid + 1;
                    }
                    j0 = lo;
                    for (int j = j0; j < ncur && cur[j].x < ea; j++) span++;
                    c = span;
                }
                const int inc = group_incl_scan(c);
                int idx = carry + inc - c;
                for (int j = j0; j < j0 + span; j++) {
                    const int2 b = cur[j];
                    const int2 v = make_int2(max(sa, b.x), min(ea, b.y));
                    if (idx < cap_row) {
                        o[idx] = v;
                        if (idx < kScanWin) wb[idx] = v;
                    }
                    idx++;
                }
                carry += group_last(inc);
            }
            cnt = carry;
        }
        cnt = (int)min((long long)cnt, cap_row);
        if (gl == 0) out_cnt[orow] = cnt;
        rout += cnt;
        // the new row becomes the current one
        if (cnt <= kScanWin) {
            wave_lds_sync();
            int2 *tmp = wa;
            wa = wb;
            wb = tmp;
            cur = wa;
        } else {
            __threadfence();
            __builtin_amdgcn_wave_barrier();
            cur = o;
        }
        ncur = cnt;
    }
    if (trace && gl == 0) trace_add(trace, rin, rout);
}

// ---------------------------------------------------------- final packing
// Runs per row of the complement of slot rows: the gaps, without an empty
// first or last one.
__global__ __launch_bounds__(256) void gap_count_kernel(RowsIn in, int R, int W, int *__restrict__ counts)
{
    const long long r = (long long)xcd_block() * 256 + threadIdx.x;
    if (r >= R) return;
    long long base;
    int n;
    row_span(in, r, base, n);
    const int *rr = in.runs + 2 * base;
    int g = n + 1;
    if (n > 0 && rr[0] == 0) g--;
    if (n > 0 && rr[2 * n - 1] == W) g--;
    counts[r] = g;
}

// Copies slot rows (or their complements) to CSR rows at row_ptr.
__global__ __launch_bounds__(256) void pack_rows_kernel(RowsIn in, int R, int W, int comp,
                                                        const int *__restrict__ row_ptr,
                                                        int *__restrict__ out_runs, long long cap,
                                                        unsigned long long *trace)
{
    const long long r = (long long)xcd_block() * kGroupsPerBlock + (threadIdx.x >> 4);
    if (r >= R) return;
    const int gl = glane();
    long long base;
    int n;
    row_span(in, r, base, n);
    const int *rr = in.runs + 2 * base;
    const long long o = row_ptr[r];
    const int nout = row_ptr[r + 1] - row_ptr[r];
    if (trace && gl == 0) trace_add(trace, (unsigned long long)n, (unsigned long long)nout);
    if ((comp ? n + 1 : n) <= kStageRuns) {
        // the whole row in registers (lane k holds runs k + 16 m)
        const int2 *r2 = (const int2 *)rr;
        const int nblk = wave_blocks(comp ? n + 1 : n);
        int2 v[kARegs];
#pragma unroll
        for (int m = 0; m < kARegs; m++) {
            if (m >= nblk) break;
            const int k = m * kGroup + gl;
            v[m] = k < n ? r2[k] : make_int2(0, 0);
        }
        const int skip = (comp && n > 0 && group_first(v[0].x) == 0) ? 1 : 0;
        int prev_end = 0;                   // end of run 16 m - 1
#pragma unroll
        for (int m = 0; m < kARegs; m++) {
            if (m * kGroup >= nout) break;
            const int k = m * kGroup + gl;
            int s, e;
            if (!comp) {
                s = v[m].x;
                e = v[m].y;
            } else if (!skip) {
                // gap k: end of run k - 1 (lane before), start of run k
                const int pe = __builtin_amdgcn_update_dpp(prev_end, v[m].y, 0x111, 0xf, 0xf, false);
                s = (k == 0) ? 0 : pe;
                e = (k == n) ? W : v[m].x;
            } else {
                // gap k + 1: end of run k, start of run k + 1 (lane after,
                // or lane 0 of the next block)
                const int nf = (m + 1 < kARegs) ? group_first(v[m + 1 < kARegs ? m + 1 : m].x) : 0;
                const int nx = __builtin_amdgcn_update_dpp(nf, v[m].x, 0x101, 0xf, 0xf, false);
                s = v[m].y;
                e = (k + 1 == n) ? W : nx;
            }
            prev_end = group_last(v[m].y);
            if (k < nout && o + k < cap) ((int2 *)out_runs)[o + k] = make_int2(s, e);
        }
        return;
    }
    const int skip = (comp && n > 0 && rr[0] == 0) ? 1 : 0;
    for (int k = gl; k < nout; k += kGroup) {
        int s, e;
        if (comp) {
            const int g = k + skip;
            s = (g == 0) ? 0 : rr[2 * g - 1];
            e = (g == n) ? W : rr[2 * g];
        } else {
            s = rr[2 * k];
            e = rr[2 * k + 1];
        }
        if (o + k < cap) ((int2 *)out_runs)[o + k] = make_int2(s, e);
    }
}

// ----------------------------------------------------- arbitrary masks on runs
// One run of a mask (section "Morphology with Arbitrary Masks", the
// run-length form): output row y of a page is the intersection of the
// accumulated row y with row y + dy of the source eroded along the line by
// the run: pixel x survives when all of x + dx .. x + dx + len - 1 are 1,
// pixels outside the line counting as 1.  A source row outside the page is
// all 1s.  With comp the source is complemented first (its gaps are the
// runs).  For the first run of a mask the accumulated row is the full row.
struct MaskRunX {
    int dx, dy, len, comp, W;
};

constexpr int kMaskBig = 1 << 30;           // stands for the infinite ends of border runs

// Candidates of a source row (n raw runs R): its runs (or gaps), a run that
// touches a border extended to infinity there, and the outside beyond each
// border as a run of its own where no run touches it.
__device__ __forceinline__ int mask_ncand(const MaskRunX &t, const int2 *R, int n)
{
    if (t.comp) return n + 1;
    return n + ((n == 0 || R[0].x != 0) ? 1 : 0) + ((n == 0 || R[n - 1].y != t.W) ? 1 : 0);
}

__device__ __forceinline__ int2 mask_cand(const MaskRunX &t, const int2 *R, int n, int k)
{
    int s, e;
    if (t.comp) {
        s = k == 0 ? -kMaskBig : R[k - 1].y;
        e = k == n ? kMaskBig : R[k].x;
    } else {
        const int i = k - ((n == 0 || R[0].x != 0) ? 1 : 0);
        if (i < 0) {
            s = -kMaskBig;
            e = 0;
        } else if (i == n) {
            s = t.W;
            e = kMaskBig;
        } else {
            s = R[i].x == 0 ? -kMaskBig : R[i].x;
            e = R[i].y == t.W ? kMaskBig : R[i].y;
        }
    }
    return make_int2(max(0, s - t.dx), min(t.W, e - t.dx - t.len + 1));
}

// Intersection of the accumulated row A (na runs) with the candidates of
// the source row (nb of them, ascending starts and ends, dead ones with
// s >= e skipped), lanes over A: bisection for the first candidate ending
// after each run's start, the overlaps counted, a group scan, then emitted.
template <class GetB>
__device__ __forceinline__ int mask_intersect(const int2 *A, int na, int nb, GetB getB, int2 *o,
                                              long long cap_row)
{
    const int gl = glane();
    int carry = 0;
    for (int k0 = 0; k0 < na; k0 += kGroup) {
        const int k = k0 + gl;
        int c = 0, span = 0, j0 = 0, sa = 0, ea = 0;
        if (k < na) {
            const int2 a = A[k];
            sa = a.x;
            ea = a.y;
            int lo = 0, hi = nb;            // the first candidate that ends after sa
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (getB(mid).y > sa) hi = mid; else lo = mid + 1;
            }
            j0 = lo;
            for (int j = j0; j < nb; j++) {
                const int2 b = getB(j);
                if (b.x >= ea) break;
                span++;
                c += live(b) ? 1 : 0;
            }
        }
        const int inc = group_incl_scan(c);
        int idx = carry + inc - c;
        for (int j = j0; j < j0 + span; j++) {
            const int2 b = getB(j);
            if (!live(b)) continue;
            if (idx < cap_row) o[idx] = make_int2(max(sa, b.x), min(ea, b.y));
            idx++;
        }
        carry += group_last(inc);
    }
    return carry;
}

__global__ __launch_bounds__(256) void mask_and_kernel(RowsIn src, int P, int H, MaskRunX t, int first,
                                                       const int *__restrict__ acc_cnt,
                                                       const int *__restrict__ acc_runs, long long cap_row,
                                                       int *__restrict__ out_cnt, int *__restrict__ out_runs,
                                                       unsigned long long *trace)
{
    __shared__ int2 stage[kGroupsPerBlock][kStageRuns];
    const long long r = (long long)xcd_block() * kGroupsPerBlock + (threadIdx.x >> 4);
    if (r >= (long long)P * H) return;      // whole group
    const int gl = glane();
    const int page = (int)(r / H), y = (int)(r - (long long)page * H), ys = y + t.dy;
    const bool outside = ys < 0 || ys >= H;
    long long base = 0;
    int n = 0;
    if (!outside) row_span(src, (long long)page * H + ys, base, n);
    const int2 *R = reinterpret_cast<const int2 *>(src.runs) + base;
    const int nb = outside ? 1 : mask_ncand(t, R, n);
    auto candB = [&](int k) { return outside ? make_int2(0, t.W) : mask_cand(t, R, n, k); };
    int2 *o = reinterpret_cast<int2 *>(out_runs) + r * cap_row;
    int carry = 0;
    if (first) {                            // the live candidates, compacted
        for (int k0 = 0; k0 < nb; k0 += kGroup) {
            const int k = k0 + gl;
            int2 c = make_int2(0, 0);
            if (k < nb) c = candB(k);
            const int l = live(c) ? 1 : 0;
            const int inc = group_incl_scan(l);
            const int idx = carry + inc - l;
            if (l && idx < cap_row) o[idx] = c;
            carry += group_last(inc);
        }
    } else {
        const int2 *A = reinterpret_cast<const int2 *>(acc_runs) + r * cap_row;
        const int na = min(max(acc_cnt[r], 0), (int)cap_row);
        if (na == 0) {
            carry = 0;                      // nothing left to intersect (erosion empties rows fast)
        } else if (nb <= kStageRuns) {
            // the source row's candidates computed once into this group's
            // LDS window: the bisections then read LDS, not global memory
            int2 *sB = stage[threadIdx.x >> 4];
            for (int k = gl; k < nb; k += kGroup) sB[k] = candB(k);
            wave_lds_sync();
            carry = mask_intersect(A, na, nb, [&](int j) { return sB[j]; }, o, cap_row);
        } else {
            carry = mask_intersect(A, na, nb, candB, o, cap_row);
        }
    }
    if (gl == 0) {
        out_cnt[r] = (int)min((long long)carry, cap_row);
        if (trace) trace_add(trace, (unsigned long long)n, (unsigned long long)carry);
    }
}

// ---------------------------------------------------------- line shifts, runs
// Every line moves right by its own shift: its runs move, are cut to the
// destination width and, with fill, the pixels that come from outside the
// source line are 1 (a run touching a source border then reaches out to
// the destination's edge).  Two passes with one group per row: counts,
// then the runs at scanned offsets.
__device__ __forceinline__ int shift_ncand(const int2 *R, int n, int Ws, int fill)
{
    if (!fill) return n;
    return n + ((n == 0 || R[0].x != 0) ? 1 : 0) + ((n == 0 || R[n - 1].y != Ws) ? 1 : 0);
}

__device__ __forceinline__ int2 shift_cand(const int2 *R, int n, int Ws, int Wd, int fill, long long sh, int k)
{
    long long s, e;
    if (!fill) {
        s = R[k].x;
        e = R[k].y;
    } else {
        const int i = k - ((n == 0 || R[0].x != 0) ? 1 : 0);
        if (i < 0) {
            s = -(1LL << 40);
            e = 0;
        } else if (i == n) {
            s = Ws;
            e = 1LL << 40;
        } else {
            s = R[i].x == 0 ? -(1LL << 40) : R[i].x;
            e = R[i].y == Ws ? (1LL << 40) : R[i].y;
        }
    }
    return make_int2((int)max(0LL, s + sh), (int)min((long long)Wd, e + sh));
}

template <bool EMIT>
__global__ __launch_bounds__(256) void shift_rows_rle_kernel(RowsIn src, long long R, int Ws, int Wd,
                                                             const int *__restrict__ shifts, int fill,
                                                             int *__restrict__ counts, const int *__restrict__ out_rp,
                                                             int *__restrict__ out_runs, long long cap,
                                                             unsigned long long *trace)
{
    const long long r = (long long)xcd_block() * kGroupsPerBlock + (threadIdx.x >> 4);
    if (r >= R) return;                     // whole group
    const int gl = glane();
    long long base;
    int n;
    row_span(src, r, base, n);
    const int2 *Rw = reinterpret_cast<const int2 *>(src.runs) + base;
    const long long sh = min(max((long long)shifts[r], -(1LL << 30)), 1LL << 30);
    const int nc = shift_ncand(Rw, n, Ws, fill);
    long long o = EMIT ? out_rp[r] : 0;
    int carry = 0;
    for (int k0 = 0; k0 < nc; k0 += kGroup) {
        const int k = k0 + gl;
        int2 c = make_int2(0, 0);
        if (k < nc) c = shift_cand(Rw, n, Ws, Wd, fill, sh, k);
        const int l = live(c) ? 1 : 0;
        const int inc = group_incl_scan(l);
        if (EMIT && l) {
            const long long idx = o + carry + inc - l;
            if (idx < cap) reinterpret_cast<int2 *>(out_runs)[idx] = c;
        }
        carry += group_last(inc);
    }
    if (gl == 0) {
        if (!EMIT) counts[r] = carry;
        if (EMIT && trace) trace_add(trace, (unsigned long long)n, (unsigned long long)carry);
    }
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
hipError_t exclusive_scan(const int *in, int n, int *out, int *tmp, hipStream_t s)
{
    if (n == 0) {
        hipLaunchKernelGGL(zero_one_kernel, dim3(1), dim3(64), 0, s, out);
        return hipGetLastError();
    }
    if (n <= kScanSingleMax) {
        hipLaunchKernelGGL(scan_single_kernel, dim3(1), dim3(kScanThreads), 0, s, in, n, out);
        return hipGetLastError();
    }
    const unsigned nb = blocks_for(n, kScanBlock);
    hipLaunchKernelGGL(scan_up_kernel, dim3(nb), dim3(kScanThreads), 0, s, in, n, tmp);
    hipLaunchKernelGGL(scan_mid_kernel, dim3(1), dim3(kScanThreads), 0, s, tmp, (int)nb);
    hipLaunchKernelGGL(scan_down_kernel, dim3(nb), dim3(kScanThreads), 0, s, in, n, tmp, out);
    return hipGetLastError();
}

static size_t r256(size_t b) { return (b + 255) & ~(size_t)255; }

// This kernel's block of trace counters (nullptr when tracing is off).
static unsigned long long *trace_block(unsigned long long *tr, int kernel)
{
    return tr ? tr + (long long)kernel * 2 * kTraceSlots * kTraceStride : nullptr;
}

hipError_t rle_from_packed(const morph_rle_t &dst, const morph_bitmap_t &src, void *ws, hipStream_t s,
                           bool traced)
{
    const int R = src.height * src.npages;
    const int nw = (src.width + 63) / 64;
    const uint64_t pad = (src.width % 64) ? ((1ull << (src.width % 64)) - 1) : ~0ull;
    int *counts = (int *)ws;
    int *tmp = (int *)((char *)ws + r256((size_t)R * sizeof(int)));
    const long long pw = (long long)src.stride_words * src.height;
    const unsigned g = blocks_for(R, kRowWaves);
    unsigned long long *tr = traced ? trace_counters() : nullptr;
    if (traced) trace_before(MORPH_K_PACK_TO_RLE, s);
    const bool narrow = nw <= kNarrowRowWords;
    const unsigned gg = blocks_for(R, kGroupsPerBlock);
    if (narrow)
        hipLaunchKernelGGL((pack_to_rle_group_kernel<false>), dim3(gg), dim3(256), 0, s, src.words, nw,
                           src.stride_words, src.height, R, pw, pad, counts, nullptr, nullptr, 0LL, nullptr);
    else
        hipLaunchKernelGGL((pack_to_rle_kernel<false>), dim3(g), dim3(64 * kRowWaves), 0, s, src.words, nw,
                           src.stride_words, src.height, R, pw, pad, counts, nullptr, nullptr, 0LL, nullptr);
    hipError_t e = exclusive_scan(counts, R, dst.row_ptr, tmp, s);
    if (e != hipSuccess) return e;
    if (narrow)
        hipLaunchKernelGGL((pack_to_rle_group_kernel<true>), dim3(gg), dim3(256), 0, s, src.words, nw,
                           src.stride_words, src.height, R, pw, pad, nullptr, dst.row_ptr, dst.runs,
                           (long long)dst.capacity, trace_block(tr, MORPH_K_PACK_TO_RLE));
    else
        hipLaunchKernelGGL((pack_to_rle_kernel<true>), dim3(g), dim3(64 * kRowWaves), 0, s, src.words, nw,
                           src.stride_words, src.height, R, pw, pad, nullptr, dst.row_ptr, dst.runs,
                           (long long)dst.capacity, trace_block(tr, MORPH_K_PACK_TO_RLE));
    if (traced) trace_after(MORPH_K_PACK_TO_RLE, s, 8.0 * nw * R + 4.0 * (R + 1));
    return hipGetLastError();
}

hipError_t rle_to_packed(const morph_bitmap_t &dst, const morph_rle_t &src, hipStream_t s)
{
    const int R = src.height * src.npages;
    const int nw = (src.width + 63) / 64;
    unsigned long long *tr = trace_counters();
    trace_before(MORPH_K_RLE_TO_PACK, s);
    if ((long long)R * nw >= 0xffffffffLL) return hipErrorInvalidValue;
    if (nw <= kNarrowRowWords)
        hipLaunchKernelGGL(rle_to_pack_group_kernel, dim3(blocks_for(R, kGroupsPerBlock)), dim3(256), 0, s,
                           src.row_ptr, src.runs, nw, R, src.height, src.width, dst.words, dst.stride_words,
                           (long long)dst.stride_words * dst.height, (long long)src.capacity,
                           LineOp{kLineNone, 1, 0, 0}, trace_block(tr, MORPH_K_RLE_TO_PACK));
    else
        hipLaunchKernelGGL(rle_to_pack_kernel, dim3(blocks_for((long long)R * nw, 256)), dim3(256), 0, s,
                           src.row_ptr, src.runs, nw, R, src.height, dst.words, dst.stride_words,
                           (long long)dst.stride_words * dst.height, (long long)src.capacity,
                           trace_block(tr, MORPH_K_RLE_TO_PACK));
    trace_after(MORPH_K_RLE_TO_PACK, s, 8.0 * nw * R + 4.0 * (R + 1));
    return hipGetLastError();
}

size_t transposed_rle_workspace(int W, int H, int P)
{
    const long long R = (long long)W * P;
    return r256((size_t)R * transpose_pieces(H) * 4) + r256((size_t)R * 4) + r256(scan_workspace(R));
}

hipError_t rle_from_packed_transposed(const morph_rle_t &dst, const morph_bitmap_t &src, uint64_t *tbuf, void *ws,
                                      hipStream_t s)
{
    const int W = src.width, H = src.height, P = src.npages;
    const long long R = (long long)W * P;
    const int np = transpose_pieces(H), nwt = (H + 63) / 64;
    if (R <= 0) return hipSuccess;
    if (R >= 0x7fffffffLL || nwt > kNarrowRowWords) return hipErrorInvalidValue;
    int *pieces = (int *)ws;
    int *cnt = (int *)((char *)ws + r256((size_t)R * np * 4));
    int *tmp = (int *)((char *)cnt + r256((size_t)R * 4));
    const morph_bitmap_t T{tbuf, H, W, nwt, P};
    unsigned long long *tr = trace_counters();
    trace_before(MORPH_K_TRANSPOSE_TO_RLE, s);
    hipError_t e = packed_transpose_counted(T, src, pieces, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(piece_sum_kernel, dim3(blocks_for(R, 256)), dim3(256), 0, s, pieces, np, R, cnt);
    e = exclusive_scan(cnt, (int)R, dst.row_ptr, tmp, s);
    if (e != hipSuccess) return e;
    const uint64_t pad = (H % 64) ? ((1ull << (H % 64)) - 1) : ~0ull;
    hipLaunchKernelGGL((pack_to_rle_group_kernel<true>), dim3(blocks_for(R, kGroupsPerBlock)), dim3(256), 0, s,
                       T.words, nwt, nwt, W, (int)R, (long long)nwt * W, pad, nullptr, dst.row_ptr, dst.runs,
                       (long long)dst.capacity, trace_block(tr, MORPH_K_TRANSPOSE_TO_RLE));
    // algorithmic: the page read, the transpose written and read back, the
    // row offsets (the runs written come from the run counters)
    trace_after(MORPH_K_TRANSPOSE_TO_RLE, s,
                8.0 * P * ((double)((W + 63) / 64) * H + 2.0 * nwt * W) + 4.0 * ((double)R + 1));
    return hipGetLastError();
}

hipError_t rle_decode_rows(const morph_bitmap_t &dst, const morph_rle_t &src, LineOp op, hipStream_t s)
{
    const int W = src.width, H = src.height, R = H * src.npages;
    const int nw = (W + 63) / 64;
    if (nw > kNarrowRowWords) return hipErrorInvalidValue;
    unsigned long long *tr = trace_counters();
    trace_before(MORPH_K_DECODE_T, s);
    hipLaunchKernelGGL(rle_to_pack_group_kernel, dim3(blocks_for(R, kGroupsPerBlock)), dim3(256), 0, s,
                       src.row_ptr, src.runs, nw, R, H, W, dst.words, dst.stride_words,
                       (long long)dst.stride_words * H, (long long)src.capacity, op,
                       trace_block(tr, MORPH_K_DECODE_T));
    trace_after(MORPH_K_DECODE_T, s, 8.0 * (double)nw * R + 4.0 * ((double)R + 1));
    return hipGetLastError();
}

hipError_t rle_decode_transposed(const morph_bitmap_t &dst, const morph_rle_t &src, LineOp op,
                                 hipStream_t s, uint64_t *tmp)
{
    const int W = src.width, H = src.height;
    const int nw = (W + 63) / 64, nk = (H + 63) / 64;
    if (tmp && nw <= kNarrowRowWords) {
        // rows of up to 128 words: decoded with the operation into tmp in
        // their own orientation, one group per row, then turned by the
        // 64 x 64 bit-block transpose; both passes run near the memory's
        // pace, where decoding straight into the transposed image streams
        // each row's runs through one lane
        const morph_bitmap_t T{tmp, W, H, nw, src.npages};
        hipError_t e = rle_decode_rows(T, src, op, s);
        if (e != hipSuccess) return e;
        return packed_transpose(dst, T, s);
    }
    const int nstrips = (nw + kDecodeStrip - 1) / kDecodeStrip;
    const int kgroups = (nk + kDecodeWaves - 1) / kDecodeWaves;
    const long long total = (long long)nstrips * kgroups * src.npages;
    if (total <= 0) return hipSuccess;
    const long long blocks = total;
    if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
    unsigned long long *tr = trace_counters();
    trace_before(MORPH_K_DECODE_T, s);
    hipLaunchKernelGGL(decode_transpose_kernel, dim3((unsigned)blocks), dim3(64 * kDecodeWaves), 0, s,
                       src.row_ptr, src.runs, (long long)src.capacity, W, H, nw, nk, nstrips, kgroups, total, dst.words,
                       dst.stride_words, (long long)dst.stride_words * W, op,
                       trace_block(tr, MORPH_K_DECODE_T));
    trace_after(MORPH_K_DECODE_T, s, 8.0 * (double)nk * W * src.npages + 4.0 * ((double)H * src.npages + 1));
    return hipGetLastError();
}

// Workspace of a run-length rectangle operation on P pages of H rows: two
// slot buffers (counts + runs) for every row the passes produce, the counts
// of the final rows, and scan scratch.
struct RleWs {
    int *cnt[2];
    int *runs[2];
    int *fcount;
    int *tmp;
    long long rows_max, cap_row;
    size_t bytes;
};

// Elements at least this tall (and wider than a column) may run between
// lines as block prefix scans (two launches) instead of the doubling steps
// (one launch per offset).
constexpr int kScanMinH = 9;
// ... and only over stacks of at least this many rows: a walk is h steps
// long, so on a few pages the doubling steps finish sooner.
constexpr long long kScanMinRows = 32768;

bool rle_uses_scan(morph_se_t se) { return se.h >= kScanMinH && se.w > 1; }

static RleWs rle_layout(void *base, int32_t W, int32_t rows, int32_t H, morph_se_t se)
{
    const long long P = rows / H;
    RleWs L{};
    // the scans keep 2 (H + h - 1) rows per page
    L.rows_max = P * (H + (long long)se.h - 1) * (rle_uses_scan(se) ? 2 : 1);
    L.cap_row = ((W + 1) / 2 + 15) & ~15LL;      // slot rows start on 128-byte lines
    char *p = (char *)base;
    size_t off = 0;
    auto take = [&](size_t b) { int *q = p ? (int *)(p + off) : nullptr; off += r256(b); return q; };
    for (int i = 0; i < 2; i++) {
        L.cnt[i] = take((size_t)L.rows_max * 4);
        L.runs[i] = take((size_t)L.rows_max * L.cap_row * 8);
    }
    L.fcount = take((size_t)P * H * 4);
    L.tmp = take(scan_workspace(P * H));
    L.bytes = off;
    return L;
}

size_t rle_op_workspace(int op, int32_t W, int32_t rows, int32_t H, morph_se_t se)
{
    (void)op;
    return rle_layout(nullptr, W, rows, H, se).bytes;
}

static RowsIn slot_rows(const RleWs &L, int i)
{
    return RowsIn{nullptr, L.cnt[i], L.runs[i], L.cap_row};
}

// Erosion of P pages (or of their complements, comp_in) by the rectangle
// (w, h, cx, cy) into slot buffer `to` and the other one, alternating.  With
// h = 1 it is the within-line pass alone.  Otherwise the first doubling step
// between lines reads `in` itself and applies the within-line pass to each
// row as it reads it; the other steps follow.  Returns the buffer that holds
// the P*H result rows.  `in` may be the other slot buffer, never `to`.
static int erode_chain(const RowsIn &in, int comp_in, int P, int W, int H, int w, int h, int cx, int cy,
                       const RleWs &L, int to, hipStream_t s, hipError_t *err, int *gap_out = nullptr,
                       bool *gaps_done = nullptr, bool scan = false)
{
    if (gaps_done) *gaps_done = false;
    const int R = P * H;
    unsigned long long *tr = trace_counters();
    if (h == 1) {
        trace_before(MORPH_K_ROW_ERODE, s);
        hipLaunchKernelGGL(row_erode_kernel, dim3(blocks_for(R, kGroupsPerBlock)), dim3(256), 0, s, in, R, W, w,
                           cx, comp_in, 0, L.cnt[to], L.runs[to], (long long)L.cap_row,
                           trace_block(tr, MORPH_K_ROW_ERODE));
        trace_after(MORPH_K_ROW_ERODE, s, 8.0 * R);
        *err = hipGetLastError();
        return to;
    }
    const RowX xs{cx, w - 1 - cx, comp_in, W};
    if (scan && rle_uses_scan(morph_se_t{w, h, cx, cy}) && (long long)P * H >= kScanMinRows) {
        const int NA = H + h - 1, nblk = (NA + h - 1) / h;
        trace_before(MORPH_K_COL_SCAN, s);
        hipLaunchKernelGGL(col_scan_kernel<true>, dim3(blocks_for((long long)P * nblk * 2, kGroupsPerBlock)),
                           dim3(256), 0, s, in, cy, H, NA, h, nblk, P, W, xs, L.cnt[to], L.runs[to],
                           (long long)L.cap_row, trace_block(tr, MORPH_K_COL_SCAN));
        trace_after(MORPH_K_COL_SCAN, s, 4.0 * P * ((double)H + 2.0 * NA));
        const int fin = 1 - to;
        trace_before(MORPH_K_COL_AND, s);
        hipLaunchKernelGGL(col_and_kernel<false>, dim3(blocks_for((long long)P * H, kGroupsPerBlock)), dim3(256), 0, s,
                           slot_rows(L, to), 0, 2 * NA, 2 * NA, NA + h - 1, div_by((unsigned)(NA - h + 1)), P, W, xs,
                           L.cnt[fin], L.runs[fin],
                           (long long)L.cap_row, gap_out, trace_block(tr, MORPH_K_COL_AND));
        trace_after(MORPH_K_COL_AND, s, 4.0 * P * (2.0 * NA + H));
        if (gap_out && gaps_done) *gaps_done = true;
        *err = hipGetLastError();
        return fin;
    }
    // rows of the extended page: 0 .. H+h-2, row x being image row x - cy
    int off = cy, real = H, NA = H + h - 1;
    int m = 1;
    int offs[40], n = 0;
    while (2 * m <= h) { offs[n++] = m; m *= 2; }
    if (h > m) offs[n++] = h - m;
    const RowX x{cx, w - 1 - cx, comp_in, W};
    int cur = -1;                           // -1: the input rows
    for (int k = 0; k < n; k++) {
        const int K = offs[k], NB = NA - K;
        const int nxt = cur < 0 ? to : 1 - cur;
        const dim3 grid(blocks_for((long long)P * NB, kGroupsPerBlock));
        int *gaps = (k == n - 1) ? gap_out : nullptr;   // the last step counts the complement's runs
        trace_before(MORPH_K_COL_AND, s);
        if (cur < 0)
            hipLaunchKernelGGL(col_and_kernel<true>, grid, dim3(256), 0, s, in, off, real, NA, K, div_by((unsigned)NB),
                               P, W, x,
                               L.cnt[nxt], L.runs[nxt], (long long)L.cap_row, gaps,
                               trace_block(tr, MORPH_K_COL_AND));
        else
            hipLaunchKernelGGL(col_and_kernel<false>, grid, dim3(256), 0, s, slot_rows(L, cur), off, real, NA, K,
                               div_by((unsigned)NB), P, W, x, L.cnt[nxt], L.runs[nxt], (long long)L.cap_row, gaps,
                               trace_block(tr, MORPH_K_COL_AND));
        if (gaps && gaps_done) *gaps_done = true;
        trace_after(MORPH_K_COL_AND, s, 4.0 * P * ((double)real + NB));
        cur = nxt;
        off = 0;
        real = NB;
        NA = NB;
    }
    *err = hipGetLastError();
    return cur;
}

// Packs the P*H slot rows of buffer b (complemented when comp) into dst.
// With gaps_done the complement's counts are already in L.fcount.
static hipError_t finish(const RleWs &L, int b, int comp, const morph_rle_t &dst, int W, hipStream_t s,
                         bool gaps_done)
{
    const int R = dst.height * dst.npages;
    const int *counts = comp ? L.fcount : L.cnt[b];
    unsigned long long *tr = trace_counters();
    trace_before(MORPH_K_PACK_ROWS, s);
    if (comp && !gaps_done) {
        hipLaunchKernelGGL(gap_count_kernel, dim3(blocks_for(R, 256)), dim3(256), 0, s, slot_rows(L, b), R, W,
                           L.fcount);
    }
    hipError_t e = exclusive_scan(counts, R, dst.row_ptr, L.tmp, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(pack_rows_kernel, dim3(blocks_for(R, kGroupsPerBlock)), dim3(256), 0, s, slot_rows(L, b), R,
                       W, comp, dst.row_ptr, dst.runs, (long long)dst.capacity,
                       trace_block(tr, MORPH_K_PACK_ROWS));
    trace_after(MORPH_K_PACK_ROWS, s, 4.0 * R + 4.0 * (R + 1));
    return hipGetLastError();
}

// erode:  E_B(A)
// dilate: not E_B^(not A)             (dilation by complementation)
// open:   not E_B^(not E_B(A))
// close:  E_B(not E_B^(not A))
hipError_t rle_rect_op(int op, const morph_rle_t &dst, const morph_rle_t &src, morph_se_t se,
                       void *ws, size_t ws_bytes, hipStream_t s)
{
    (void)ws_bytes;
    const int P = src.npages, H = src.height, W = src.width;
    const RleWs L = rle_layout(ws, W, P * H, H, se);
    const RowsIn in{src.row_ptr, nullptr, src.runs, (long long)src.capacity};
    const int w = se.w, h = se.h, cx = se.cx, cy = se.cy;
    const int rx = w - 1 - cx, ry = h - 1 - cy;
    hipError_t e = hipSuccess;
    bool g = false;                 // the complement's counts came with the last step
    int b;
    // The block scans pay off where the rows they intersect thin out: the
    // erosion of the image by an element wider than a column, and the second
    // chain of an opening or closing by one (the complement of an eroded or
    // dilated image has few runs).  Eroding the complement of the image
    // itself keeps its long white runs through every step, and a single
    // column leaves the rows as they are; there the doubling steps are
    // faster (measured on the letter batch).
    const bool wide = w > 1;
    if (h == 1 && (op == MORPH_OPEN || op == MORPH_CLOSE)) {
        // one row: the opening keeps the runs whose erosion is not empty,
        // unchanged, in one pass; the closing does the same to the gaps with
        // the reflected origin and takes the complement
        const int comp = op == MORPH_CLOSE ? 1 : 0;
        const int R = P * H;
        unsigned long long *tr = trace_counters();
        trace_before(MORPH_K_ROW_ERODE, s);
        hipLaunchKernelGGL(row_erode_kernel, dim3(blocks_for(R, kGroupsPerBlock)), dim3(256), 0, s, in, R, W, w,
                           comp ? rx : cx, comp, 1, L.cnt[0], L.runs[0], (long long)L.cap_row,
                           trace_block(tr, MORPH_K_ROW_ERODE));
        trace_after(MORPH_K_ROW_ERODE, s, 8.0 * R);
        e = hipGetLastError();
        return e != hipSuccess ? e : finish(L, 0, comp, dst, W, s, false);
    }
    switch (op) {
    case MORPH_ERODE:
        b = erode_chain(in, 0, P, W, H, w, h, cx, cy, L, 0, s, &e, nullptr, nullptr, wide);
        return e != hipSuccess ? e : finish(L, b, 0, dst, W, s, false);
    case MORPH_DILATE:
        b = erode_chain(in, 1, P, W, H, w, h, rx, ry, L, 0, s, &e, L.fcount, &g);
        return e != hipSuccess ? e : finish(L, b, 1, dst, W, s, g);
    case MORPH_OPEN:
        b = erode_chain(in, 0, P, W, H, w, h, cx, cy, L, 0, s, &e, nullptr, nullptr, wide);
        if (e != hipSuccess) return e;
        b = erode_chain(slot_rows(L, b), 1, P, W, H, w, h, rx, ry, L, 1 - b, s, &e, L.fcount, &g, wide);
        return e != hipSuccess ? e : finish(L, b, 1, dst, W, s, g);
    case MORPH_CLOSE:
        b = erode_chain(in, 1, P, W, H, w, h, rx, ry, L, 0, s, &e);
        if (e != hipSuccess) return e;
        b = erode_chain(slot_rows(L, b), 1, P, W, H, w, h, cx, cy, L, 1 - b, s, &e, nullptr, nullptr, wide);
        return e != hipSuccess ? e : finish(L, b, 0, dst, W, s, false);
    }
    return hipErrorInvalidValue;
}

// ------------------------------------------------------ masks: host side
// Workspace: three slot buffers (the accumulator alternates between two
// that are not the chain's input), the final counts and scan scratch.
struct MaskWs {
    int *cnt[3];
    int *runs[3];
    int *fcount, *tmp;
    long long cap_row;
    size_t bytes;
};

static MaskWs mask_layout(void *base, int W, long long R)
{
    MaskWs L{};
    L.cap_row = ((W + 1) / 2 + 15) & ~15LL;
    char *p = (char *)base;
    size_t off = 0;
    auto take = [&](size_t b) { int *q = p ? (int *)(p + off) : nullptr; off += r256(b); return q; };
    for (int i = 0; i < 3; i++) {
        L.cnt[i] = take((size_t)R * 4);
        L.runs[i] = take((size_t)R * L.cap_row * 8);
    }
    L.fcount = take((size_t)R * 4);
    L.tmp = take(scan_workspace(R));
    L.bytes = off;
    return L;
}

size_t rle_mask_workspace(int W, long long R) { return mask_layout(nullptr, W, R).bytes; }

// Erosion of P pages (or of their complements) by the mask runs m, into the
// slot buffers other than `avoid`; returns the buffer with the result.
static int mask_chain(const RowsIn &in, int comp, const MaskRunsArg &m, int P, int W, int H, const MaskWs &L,
                      int avoid, hipStream_t s, hipError_t *err)
{
    const long long R = (long long)P * H;
    unsigned long long *tr = trace_counters();
    const int n = std::max(m.n, 1);
    int cur = -1;
    for (int q = 0; q < n; q++) {
        int nxt = 0;
        while (nxt == avoid || nxt == cur) nxt++;
        // the empty mask: one pseudo-run whose source rows all lie outside
        const MaskRunX t = m.n ? MaskRunX{m.dx[q], m.dy[q], m.len[q], comp, W} : MaskRunX{0, H, 1, comp, W};
        trace_before(MORPH_K_MASK_RLE, s);
        hipLaunchKernelGGL(mask_and_kernel, dim3(blocks_for(R, kGroupsPerBlock)), dim3(256), 0, s, in, P, H, t,
                           q == 0 ? 1 : 0, cur < 0 ? nullptr : L.cnt[cur], cur < 0 ? nullptr : L.runs[cur],
                           (long long)L.cap_row, L.cnt[nxt], L.runs[nxt], trace_block(tr, MORPH_K_MASK_RLE));
        trace_after(MORPH_K_MASK_RLE, s, 4.0 * R * (q == 0 ? 1 : 2));
        cur = nxt;
    }
    *err = hipGetLastError();
    return cur;
}

// erode: E_M(A); dilate: not E_M^(not A); open, close composed (the
// reflected runs mr are those of the reflected mask).
hipError_t rle_mask_op(int op, const morph_rle_t &dst, const morph_rle_t &src, const MaskRunsArg &m,
                       const MaskRunsArg &mr, void *ws, hipStream_t s)
{
    const int P = src.npages, H = src.height, W = src.width;
    const MaskWs L = mask_layout(ws, W, (long long)P * H);
    const RowsIn in{src.row_ptr, nullptr, src.runs, (long long)src.capacity};
    auto slot = [&](int i) { return RowsIn{nullptr, L.cnt[i], L.runs[i], L.cap_row}; };
    auto fin = [&](int b, int comp) {
        RleWs F{};
        F.cnt[0] = L.cnt[b];
        F.runs[0] = L.runs[b];
        F.cnt[1] = F.runs[1] = nullptr;
        F.fcount = L.fcount;
        F.tmp = L.tmp;
        F.cap_row = L.cap_row;
        return finish(F, 0, comp, dst, W, s, false);
    };
    hipError_t e = hipSuccess;
    int b;
    switch (op) {
    case MORPH_ERODE:
        b = mask_chain(in, 0, m, P, W, H, L, -1, s, &e);
        return e != hipSuccess ? e : fin(b, 0);
    case MORPH_DILATE:
        b = mask_chain(in, 1, mr, P, W, H, L, -1, s, &e);
        return e != hipSuccess ? e : fin(b, 1);
    case MORPH_OPEN:
        b = mask_chain(in, 0, m, P, W, H, L, -1, s, &e);
        if (e != hipSuccess) return e;
        b = mask_chain(slot(b), 1, mr, P, W, H, L, b, s, &e);
        return e != hipSuccess ? e : fin(b, 1);
    case MORPH_CLOSE:
        b = mask_chain(in, 1, mr, P, W, H, L, -1, s, &e);
        if (e != hipSuccess) return e;
        b = mask_chain(slot(b), 1, m, P, W, H, L, b, s, &e);
        return e != hipSuccess ? e : fin(b, 0);
    }
    return hipErrorInvalidValue;
}

size_t shift_rows_rle_workspace(long long R) { return r256((size_t)R * 4) + scan_workspace(R); }

hipError_t shift_rows_rle(const morph_rle_t &dst, const morph_rle_t &src, const int *shifts, int fill, void *ws,
                          hipStream_t s)
{
    const long long R = (long long)src.height * src.npages;
    int *counts = (int *)ws;
    int *tmp = (int *)((char *)ws + r256((size_t)R * 4));
    const RowsIn in{src.row_ptr, nullptr, src.runs, (long long)src.capacity};
    const dim3 grid(blocks_for(R, kGroupsPerBlock));
    unsigned long long *tr = trace_counters();
    trace_before(MORPH_K_SHIFT_RLE, s);
    hipLaunchKernelGGL(shift_rows_rle_kernel<false>, grid, dim3(256), 0, s, in, R, src.width, dst.width, shifts, fill,
                       counts, nullptr, nullptr, 0LL, nullptr);
    hipError_t e = exclusive_scan(counts, (int)R, dst.row_ptr, tmp, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(shift_rows_rle_kernel<true>, grid, dim3(256), 0, s, in, R, src.width, dst.width, shifts, fill,
                       nullptr, dst.row_ptr, dst.runs, (long long)dst.capacity, trace_block(tr, MORPH_K_SHIFT_RLE));
    trace_after(MORPH_K_SHIFT_RLE, s, 8.0 * R + 4.0 * (R + 1));
    return hipGetLastError();
}

// --------------------------------------------- conversion without allocation
// Scratch of the allocation-free conversion (row counts, then the scan's
// block sums): a file-scope device array that every GPU the library runs on
// holds until the process ends.  Its name is a host-side stand-in in host
// code; the device address comes from hipGetSymbolAddress, looked up once
// per device (with that device current) on the first call there, and only
// that address is ever passed to kernels.  Every call on a GPU shares the
// array: calls that overlap on one GPU race.  Nothing in it needs clearing:
// the count launch writes every row's count and the scan every block sum.
constexpr size_t kNoAllocScratchBytes = (size_t)16 << 20;
__device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_dev[kMaxDevices];

static hipError_t scratch_address(void **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_dev[dev] = p;
    }
    *out = g_scratch_dev[dev];
    return hipSuccess;
}

static_assert(((size_t)MORPH_NOALLOC_MAX_ROWS * 4 + 255) / 256 * 256 +
                  ((size_t)MORPH_NOALLOC_MAX_ROWS + kScanBlock - 1) / kScanBlock * 4 + 4 <= kNoAllocScratchBytes,
              "the fixed scratch must hold the counts and scan partials of MORPH_NOALLOC_MAX_ROWS rows");

hipError_t rle_from_packed_noalloc(const morph_rle_t &dst, const morph_bitmap_t &src, hipStream_t s)
{
    const long long R = (long long)src.height * src.npages;
    if (R > MORPH_NOALLOC_MAX_ROWS) return hipErrorInvalidValue;   // checked by the entry point first
    void *ws = nullptr;
    const hipError_t e = scratch_address(&ws);
    if (e != hipSuccess) return e;
    return rle_from_packed(dst, src, ws, s, false);
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
