// Rectangle operations on run-length images, one band of rows per
// workgroup with every intermediate row in LDS.
//
// Method (paper, section "2D Morphological Operators for Rectangular
// Masks", third strategy): within lines first -- each run (or, for a
// complemented chain, each gap) shrinks by the element's reach on either
// side unless that side is the row border (section "Within-Line
// Morphological Operations") -- then between lines: output row y of an
// erosion chain is the intersection of the h shrunk rows y - up .. y + dn,
// computed by the logarithmic decomposition (section "Efficient Binary
// Decompositions": offsets 1, 2, 4, ... then h - m), each step the
// intersection of two rows' interval lists (section "Between Line Boolean
// Operations").  Dilation, opening and closing are chains of erosions of
// complements, exactly as for the packed path.
//
// GPU form.  A workgroup owns R output rows of one page.  It loads the
// runs of the rows the band depends on (R + the vertical reach of every
// chain) straight from the CSR arrays -- one contiguous range -- shrinks
// them as it stores them in LDS, and runs every doubling step, and the
// second chain of an opening or closing, in LDS.  Candidates are packed as
// 16-bit start and end in one word.  Every pass over candidates is flat:
// the 256 threads split the pass's candidates (all rows of the band
// together) into equal contiguous chunks, so rows of any length keep every
// lane busy; a first walk counts each candidate's output (a bisection in
// the partner row for the first overlapping interval), a workgroup scan of
// the chunk totals places the output, and a second walk writes it.  Only
// the band's final rows leave LDS.
//
// The result has to land in CSR form, whose offsets depend on every row's
// count, so an operation is two launches around a scan: the count launch
// runs the band and writes each output row's run count, the scan turns the
// counts into row_ptr, and the emit launch runs the band again and writes
// the runs.  A band whose rows do not fit in LDS is retried in halves; a
// single output row that still does not fit goes to a short list, which a
// small grid of workgroups finishes with the same code on buffers in the
// caller's workspace.
#include "common.h"

#include <algorithm>

namespace morph {

namespace {

constexpr int kBT = 256;                 // threads per workgroup
constexpr int kBandCap = 5120;           // candidates per LDS buffer (3 buffers: 60 KiB)
constexpr int kBandRowsMax = 384;        // rows a band keeps in LDS (its output rows plus halos)
constexpr int kFallbackGroups = 16;      // workgroups finishing rows that do not fit in LDS

__device__ __forceinline__ unsigned pk(int s, int e) { return (unsigned)s | ((unsigned)e << 16); }
__device__ __forceinline__ int ps(unsigned v) { return (int)(v & 0xffffu); }
__device__ __forceinline__ int pe(unsigned v) { return (int)(v >> 16); }

// One erosion chain: shrink by (cx, right) along the lines, intersect the
// rows up above and dn below; comp: the chain erodes its input's complement.
struct Chain {
    int cx, right, up, dn, comp;
};

struct BandArgs {
    const int *rp;              // source CSR
    const int2 *runs;
    long long cap_in;           // runs the source array holds (offsets are clamped to it)
    int W, H, P;
    int nch;                    // 1 or 2 chains
    Chain ch[2];
    int out_comp;               // the result is the complement of the last chain's rows
    int R;                      // output rows per band
    int nbands;                 // bands per page
    // count launch
    int *counts;                // per output row
    int *defer_n, *defer_rows;  // rows left to the fallback grid
    // emit launch
    const int *out_rp;
    int2 *out_runs;
    long long cap_out;
    unsigned long long *trace;  // runs read / written (tracing on), or nullptr
};

// Where a workgroup keeps its rows: three candidate buffers of `cap`
// entries and two offset arrays of `rows_max` + 1 entries, in LDS for the
// band kernel, in the workspace for the fallback grid.
struct Bufs {
    unsigned *a, *b, *meta;
    int *offa, *offb;
    int *scan;                  // kBT + 1 ints
    int *flag;                  // a few ints
    int cap, rows_max;
};

// Exclusive scan of one int per thread over the workgroup; returns the
// thread's base and sets *total.  Two barriers.
__device__ __forceinline__ int wg_scan(int v, int *scan, int *total)
{
    const int lane = (int)(threadIdx.x & 63), wv = (int)(threadIdx.x >> 6);
    int x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) scan[wv] = x;
    __syncthreads();
    int base = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < kBT / 64; k++) {
        const int t = scan[k];
        if (k < wv) base += t;
        tot += t;
    }
    __syncthreads();
    *total = tot;
    return base + x - v;
}

// off[1..n] hold counts: turns off[0..n] into their running sums (off[0] =
// 0, off[n] = the total, returned).  Each thread sums a few consecutive
// rows, one workgroup scan places them.
__device__ int rows_prefix(int *off, int n, int *scan)
{
    const int k = (n + kBT - 1) / kBT;
    const int j0 = min(n, (int)threadIdx.x * k), j1 = min(n, j0 + k);
    int sum = 0;
    for (int j = j0; j < j1; j++) sum += off[j + 1];
    int total;
    int run = wg_scan(sum, scan, &total);        // every count is read before any is overwritten
    for (int j = j0; j < j1; j++) {
        run += off[j + 1];
        off[j + 1] = run;
    }
    if (threadIdx.x == 0) off[0] = 0;
    __syncthreads();
    return total;
}

// Smallest r in [0, n] with off[r] >= c (off ascending, off[n] >= c).
__device__ __forceinline__ int first_at_or_after(const int *off, int n, int c)
{
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (off[mid] < c) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// Offsets of the rows that start at or after the pass's end: the total.
__device__ __forceinline__ void tail_offsets(const int *raw, int n, int nraw, int *off, int total)
{
    for (int j = threadIdx.x; j <= n; j += kBT)
        if (raw[j] >= nraw) off[j] = total;
}

// Trace counters of the benchmark's byte accounting: runs read / written,
// over 256 slots of one 128-byte line each.
__device__ __forceinline__ void trace_runs(unsigned long long *tr, unsigned long long in, unsigned long long out)
{
    const int slot = (int)(blockIdx.x & 255u);
    if (in) atomicAdd(tr + (long long)slot * 16, in);
    if (out) atomicAdd(tr + (long long)(256 + slot) * 16, out);
}

// Chunk of a flat pass over n items: [c0, c1) for this thread.  Chunks are
// an odd number of items long so that the lanes' LDS addresses spread over
// the banks.
__device__ __forceinline__ void chunk_of(int n, int &c0, int &c1)
{
    int q = (n + kBT - 1) / kBT;
    if (q > 1 && !(q & 1)) q++;
    c0 = min(n, (int)threadIdx.x * q);
    c1 = min(n, c0 + q);
}

// First row r in [0, nrows] with off[r] > c, less one: the row holding c.
__device__ __forceinline__ int row_of(const int *off, int nrows, int c)
{
    int lo = 0, hi = nrows;              // off[lo] <= c < off[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (off[mid] <= c) lo = mid; else hi = mid;
    }
    return lo;
}

// ------------------------------------------------------------------ load
// The source rows of page `page`, image rows y0 .. y0 + n - 1 (rows outside
// the image are full rows: erosion sees 1 outside), as chain c's candidates:
// the runs, or with comp the gaps, shrunk by (cx, right) where that side is
// not a row border, vanished ones dropped.  Into bf.a with offsets bf.offa.
// Returns false when they do not fit.
__device__ bool load_rows(const BandArgs &A, const Chain &c, int page, int y0, int n, Bufs &bf)
{
    const int W = A.W;
    // raw candidates per row (before dropping): runs (+1 gap) or one full
    // row; the rows' first runs go to bf.offa until the second walk
    int *raw = bf.offb;                  // raw offsets, n + 1 entries
    int *first = bf.offa;
    for (int j = threadIdx.x; j < n; j += kBT) {
        const int y = y0 + j;
        int k = 1, a = 0;
        if (y >= 0 && y < A.H) {
            const long long r = (long long)page * A.H + y;
            const long long lo = min((long long)max(A.rp[r], 0), A.cap_in), hi = min((long long)A.rp[r + 1], A.cap_in);
            k = (int)max(0LL, hi - lo) + c.comp;
            a = (int)lo;
        }
        raw[j + 1] = k;
        first[j] = a;
    }
    __syncthreads();
    const int nraw = rows_prefix(raw, n, bf.scan);
    if (nraw > bf.cap) return false;
    int c0, c1;
    chunk_of(nraw, c0, c1);
    // the candidate of raw index i (row j)
    auto cand = [&](int j, int i) -> unsigned {
        const int y = y0 + j;
        if (y < 0 || y >= A.H) return pk(0, W);
        const int a = first[j];
        const int nr = raw[j + 1] - raw[j] - c.comp;
        const int k = i - raw[j];
        int s, e;
        if (c.comp) {
            s = k == 0 ? 0 : A.runs[a + k - 1].y;
            e = k == nr ? W : A.runs[a + k].x;
        } else {
            const int2 v = A.runs[a + k];
            s = v.x;
            e = v.y;
        }
        const int ns = s == 0 ? 0 : s + c.cx;
        const int ne = e == W ? W : e - c.right;
        return ns < ne ? pk(ns, ne) : 0u;
    };
    int live = 0;
    if (c0 < c1) {
        int j = row_of(raw, n, c0);
        for (int i = c0; i < c1; i++) {
            while (raw[j + 1] <= i) j++;
            const unsigned v = cand(j, i);
            bf.meta[i] = v;              // kept for the second walk
            live += (ps(v) < pe(v)) ? 1 : 0;
        }
    }
    int total;
    const int base = wg_scan(live, bf.scan, &total);
    // second walk: the live candidates, and the offset of every row that
    // starts inside this thread's chunk
    if (c0 < c1) {
        int pos = base;
        int r = first_at_or_after(raw, n, c0);
        for (int i = c0; i < c1; i++) {
            while (raw[r] == i) bf.offa[r++] = pos;       // raw[n] = nraw > i ends it
            const unsigned v = bf.meta[i];
            if (ps(v) < pe(v)) bf.a[pos++] = v;
        }
    }
    tail_offsets(raw, n, nraw, bf.offa, total);
    __syncthreads();
    return true;
}

// ------------------------------------------------------------------ step
// Rows 0 .. n-1 in (src, soff); output row i = row i AND row i + K, for
// i < n - K, into (dst, doff).  Returns false when the output does not fit.
__device__ bool and_step(const unsigned *src, const int *soff, int n, int K, unsigned *dst, int *doff,
                         unsigned *meta, Bufs &bf)
{
    const int no = n - K;
    const int na = soff[no];             // candidates of rows 0 .. no-1
    int c0, c1;
    chunk_of(na, c0, c1);
    int cnt = 0;
    if (c0 < c1) {
        int i = row_of(soff, no, c0);
        int jlo = 0;
        for (int c = c0; c < c1; c++) {
            if (soff[i + 1] <= c) {
                while (soff[i + 1] <= c) i++;
                jlo = 0;
            }
            const unsigned a = src[c];
            const int sa = ps(a), ea = pe(a);
            const int bs = soff[i + K], be = soff[i + K + 1];
            // first interval of row i + K ending after sa (ends ascend; starts
            // of row i ascend, so the bound only moves right along a row)
            int lo = max(bs, jlo), hi = be;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (pe(src[mid]) > sa) hi = mid; else lo = mid + 1;
            }
            jlo = lo;
            int q = lo;
            while (q < be && ps(src[q]) < ea) q++;
            meta[c] = (unsigned)(lo - bs) | ((unsigned)(q - lo) << 16);
            cnt += q - lo;               // every overlap of two live intervals is non-empty
        }
    }
    int total;
    const int base = wg_scan(cnt, bf.scan, &total);
    if (total > bf.cap) return false;    // uniform: every thread saw the same total
    if (c0 < c1) {
        int pos = base;
        int r = first_at_or_after(soff, no, c0);
        int i = row_of(soff, no, c0);
        for (int c = c0; c < c1; c++) {
            while (soff[r] == c) doff[r++] = pos;         // soff[no] = na > c ends it
            while (soff[i + 1] <= c) i++;
            const unsigned a = src[c];
            const int sa = ps(a), ea = pe(a);
            const unsigned m = meta[c];
            const int j0 = soff[i + K] + (int)(m & 0xffffu), span = (int)(m >> 16);
            for (int q = 0; q < span; q++) {
                const unsigned b = src[j0 + q];
                dst[pos++] = pk(max(sa, ps(b)), min(ea, pe(b)));
            }
        }
    }
    tail_offsets(soff, no, na, doff, total);
    __syncthreads();
    return true;
}

// All doubling steps of an erosion by h rows over n rows in bf.a (offsets
// bf.offa); the n - h + 1 result rows end in bf.a again.
__device__ bool chain_steps(int h, int n, Bufs &bf)
{
    int m = 1;
    while (m < h) {
        const int K = (2 * m <= h) ? m : h - m;     // 1, 2, 4, ... then the rest
        if (!and_step(bf.a, bf.offa, n, K, bf.b, bf.offb, bf.meta, bf)) return false;
        n -= K;
        unsigned *t = bf.a; bf.a = bf.b; bf.b = t;
        int *to = bf.offa; bf.offa = bf.offb; bf.offb = to;
        m = (2 * m <= h) ? 2 * m : h;
    }
    return true;
}

// The second chain's input: rows of image rows y0 .. y0 + n - 1; inside the
// image the gaps of the first chain's row (image row y - x0 of bf.a),
// shrunk; outside, full rows.  Into bf.b, then swapped into bf.a.
__device__ bool build_chain2(const BandArgs &A, const Chain &c, int y0, int n, int x0, Bufs &bf)
{
    const int W = A.W;
    int *raw = bf.offb;
    for (int j = threadIdx.x; j < n; j += kBT) {
        const int y = y0 + j;
        raw[j + 1] = (y >= 0 && y < A.H) ? bf.offa[y - x0 + 1] - bf.offa[y - x0] + 1 : 1;
    }
    __syncthreads();
    const int nraw = rows_prefix(raw, n, bf.scan);
    if (nraw > bf.cap) return false;
    int c0, c1;
    chunk_of(nraw, c0, c1);
    auto cand = [&](int j, int i) -> unsigned {
        const int y = y0 + j;
        if (y < 0 || y >= A.H) return pk(0, W);
        const int o = bf.offa[y - x0], nr = bf.offa[y - x0 + 1] - o;
        const int k = i - raw[j];
        const int s = k == 0 ? 0 : pe(bf.a[o + k - 1]);
        const int e = k == nr ? W : ps(bf.a[o + k]);
        const int ns = s == 0 ? 0 : s + c.cx;
        const int ne = e == W ? W : e - c.right;
        return ns < ne ? pk(ns, ne) : 0u;
    };
    int live = 0;
    if (c0 < c1) {
        int j = row_of(raw, n, c0);
        for (int i = c0; i < c1; i++) {
            while (raw[j + 1] <= i) j++;
            const unsigned v = cand(j, i);
            bf.meta[i] = v;
            live += (ps(v) < pe(v)) ? 1 : 0;
        }
    }
    int total;
    const int base = wg_scan(live, bf.scan, &total);
    // the first chain's rows and offsets are not read past this point: the
    // new rows go to bf.b and their offsets over bf.offa
    if (c0 < c1) {
        int pos = base;
        int r = first_at_or_after(raw, n, c0);
        for (int i = c0; i < c1; i++) {
            while (raw[r] == i) bf.offa[r++] = pos;
            const unsigned v = bf.meta[i];
            if (ps(v) < pe(v)) bf.b[pos++] = v;
        }
    }
    tail_offsets(raw, n, nraw, bf.offa, total);
    __syncthreads();
    unsigned *t = bf.a; bf.a = bf.b; bf.b = t;
    return true;
}

// ---------------------------------------------------------------- a band
// Output rows y .. y + r - 1 of page `page`.  COUNT: writes their run
// counts; EMIT: writes their runs at out_rp.  false: they do not fit.
template <bool EMIT>
__device__ bool run_band(const BandArgs &A, int page, int y, int r, Bufs &bf)
{
    const Chain &c1 = A.ch[0];
    int ya, nrows;                           // first image row held, rows held
    if (A.nch == 1) {
        ya = y - c1.up;
        nrows = r + c1.up + c1.dn;
        if (nrows > bf.rows_max) return false;
        if (!load_rows(A, c1, page, ya, nrows, bf)) return false;
        if (!chain_steps(c1.up + c1.dn + 1, nrows, bf)) return false;
    } else {
        const Chain &c2 = A.ch[1];
        // chain 2 reads image rows y - up2 .. y + r - 1 + dn2; chain 1 is
        // needed for those inside the image only
        const int z0 = max(0, y - c2.up), z1 = min(A.H, y + r + c2.dn);
        const int n2 = r + c2.up + c2.dn;
        if (n2 > bf.rows_max || z1 - z0 + c1.up + c1.dn > bf.rows_max) return false;
        if (z1 > z0) {
            if (!load_rows(A, c1, page, z0 - c1.up, z1 - z0 + c1.up + c1.dn, bf)) return false;
            if (!chain_steps(c1.up + c1.dn + 1, z1 - z0 + c1.up + c1.dn, bf)) return false;
        } else {
            if (threadIdx.x == 0) bf.offa[0] = 0;
            __syncthreads();
        }
        if (!build_chain2(A, c2, y - c2.up, n2, z0, bf)) return false;
        if (!chain_steps(c2.up + c2.dn + 1, n2, bf)) return false;
    }
    (void)ya;
    (void)nrows;
    // the r result rows are rows 0 .. r-1 of bf.a
    const int W = A.W;
    const int wv = (int)(threadIdx.x >> 6), lane = (int)(threadIdx.x & 63);
    for (int i = wv; i < r; i += kBT / 64) {
        const int o = bf.offa[i], n = bf.offa[i + 1] - o;
        const long long row = (long long)page * A.H + y + i;
        if (!A.out_comp) {
            if (!EMIT) {
                if (lane == 0) A.counts[row] = n;
            } else {
                const long long base = A.out_rp[row];
                for (int k = lane; k < n; k += 64)
                    if (base + k < A.cap_out) {
                        const unsigned v = bf.a[o + k];
                        A.out_runs[base + k] = make_int2(ps(v), pe(v));
                    }
            }
        } else {
            // the gaps: gap k lies between run k-1 and run k (borders at the
            // ends), without an empty first or last one
            const int skip = (n > 0 && ps(bf.a[o]) == 0) ? 1 : 0;
            const int ng = n + 1 - skip - ((n > 0 && pe(bf.a[o + n - 1]) == W) ? 1 : 0);
            if (!EMIT) {
                if (lane == 0) A.counts[row] = ng;
            } else {
                const long long base = A.out_rp[row];
                for (int k = lane; k < ng; k += 64) {
                    const int g = k + skip;
                    const int s = g == 0 ? 0 : pe(bf.a[o + g - 1]);
                    const int e = g == n ? W : ps(bf.a[o + g]);
                    if (base + k < A.cap_out) A.out_runs[base + k] = make_int2(s, e);
                }
            }
        }
    }
    __syncthreads();
    return true;
}

// Output rows [y0, y1) of a page: whole band first, halves on overflow; a
// single row that does not fit is left to the fallback grid (listed by the
// count launch; the emit launch reaches the same decision and skips it).
template <bool EMIT>
__device__ void run_rows(const BandArgs &A, int page, int y0, int y1, Bufs &bf)
{
    int y = y0, r = y1 - y0;
    while (y < y1) {
        r = min(r, y1 - y);
        if (run_band<EMIT>(A, page, y, r, bf)) {
            y += r;
            continue;
        }
        if (r > 1) {
            r = (r + 1) / 2;
            continue;
        }
        if (!EMIT && threadIdx.x == 0) {
            const int k = atomicAdd(A.defer_n, 1);
            A.defer_rows[k] = page * A.H + y;
        }
        y += 1;
        r = y1 - y0;
    }
}

template <bool EMIT>
__global__ __launch_bounds__(kBT) void rle_band_kernel(BandArgs A)
{
    __shared__ unsigned sa[kBandCap], sb[kBandCap], sm[kBandCap];
    __shared__ int oa[kBandRowsMax + 1], ob[kBandRowsMax + 1];
    __shared__ int scan[kBT / 64 + 1], flag[4];
    const int band = (int)xcd_block();
    if (band >= A.nbands * A.P) return;      // whole workgroup
    const int page = band / A.nbands, b = band - page * A.nbands;
    const int y0 = b * A.R, y1 = min(A.H, y0 + A.R);
    Bufs bf{sa, sb, sm, oa, ob, scan, flag, kBandCap, kBandRowsMax};
    run_rows<EMIT>(A, page, y0, y1, bf);
    if (EMIT && A.trace && threadIdx.x == 0) {
        const long long r0 = (long long)page * A.H + y0, r1 = (long long)page * A.H + y1;
        trace_runs(A.trace, (unsigned long long)max(0, A.rp[r1] - A.rp[r0]),
                   (unsigned long long)max(0, A.out_rp[r1] - A.out_rp[r0]));
    }
}

// The rows no band could fit, one at a time per workgroup, on buffers in
// the workspace large enough for any single row.
template <bool EMIT>
__global__ __launch_bounds__(kBT) void rle_band_fallback_kernel(BandArgs A, unsigned *scratch, long long cap,
                                                                int rows_max)
{
    __shared__ int scan[kBT / 64 + 1], flag[4];
    const int n = *A.defer_n;
    unsigned *base = scratch + (size_t)blockIdx.x * (3 * (size_t)cap + 2 * ((size_t)rows_max + 1));
    Bufs bf{base, base + cap, base + 2 * cap, (int *)(base + 3 * cap), (int *)(base + 3 * cap) + rows_max + 1,
            scan, flag, (int)cap, rows_max};
    for (int k = blockIdx.x; k < n; k += gridDim.x) {
        const int row = A.defer_rows[k];
        const int page = row / A.H, y = row - page * A.H;
        Bufs b2 = bf;
        // buffers sized for any canonical row: a failure here means a
        // malformed input; its row is left empty
        if (!run_band<EMIT>(A, page, y, 1, b2) && !EMIT && threadIdx.x == 0) A.counts[row] = 0;
        if (EMIT && A.trace && threadIdx.x == 0)
            trace_runs(A.trace, (unsigned long long)max(0, A.rp[row + 1] - A.rp[row]),
                       (unsigned long long)max(0, A.out_rp[row + 1] - A.out_rp[row]));
    }
}

__global__ void clear_one_kernel(int *p)
{
    if (threadIdx.x == 0) *p = 0;
}

}  // namespace

// ----------------------------------------------------------------- host
// The chains of each operation (dilation = complement of the erosion of the
// complement by the reflected element).
static int band_chains(int op, morph_se_t se, Chain (&ch)[2], int &out_comp)
{
    const int rx = se.w - 1 - se.cx, ry = se.h - 1 - se.cy;
    const Chain B{se.cx, rx, se.cy, ry, 0}, Bc{se.cx, rx, se.cy, ry, 1}, Rc{rx, se.cx, ry, se.cy, 1};
    switch (op) {
    case MORPH_ERODE: ch[0] = B; out_comp = 0; return 1;
    case MORPH_DILATE: ch[0] = Rc; out_comp = 1; return 1;
    case MORPH_OPEN: ch[0] = B; ch[1] = Rc; out_comp = 1; return 2;
    default: ch[0] = Rc; ch[1] = Bc; out_comp = 0; return 2;
    }
}

static int band_halo(int op, morph_se_t se)
{
    return (op == MORPH_OPEN || op == MORPH_CLOSE ? 2 : 1) * (se.h - 1);
}

bool rle_band_applies(int op, int32_t W, morph_se_t se)
{
    return W >= 1 && W < 65536 && band_halo(op, se) + 1 <= kBandRowsMax;
}

static size_t r256b(size_t b) { return (b + 255) & ~(size_t)255; }

// Workspace: row counts, scan scratch, the deferred-row list and the
// fallback grid's buffers (sized for one output row of any content).
struct BandWs {
    size_t counts, tmp, defer, fb, total;
    long long fb_cap;
    int fb_rows;
};

static BandWs band_ws(int op, int32_t W, long long rows, morph_se_t se)
{
    BandWs w{};
    w.counts = r256b((size_t)rows * 4);
    w.tmp = r256b(scan_workspace(rows));
    w.defer = r256b((size_t)(rows + 1) * 4);
    w.fb_rows = band_halo(op, se) + 1;
    w.fb_cap = (long long)w.fb_rows * ((W + 1) / 2 + 2);
    w.fb = r256b((size_t)kFallbackGroups * (3 * (size_t)w.fb_cap + 2 * ((size_t)w.fb_rows + 1)) * 4);
    w.total = w.counts + w.tmp + w.defer + w.fb;
    return w;
}

size_t rle_band_workspace(int op, int32_t W, long long rows, morph_se_t se)
{
    return band_ws(op, W, rows, se).total;
}

hipError_t rle_band_op(int op, const morph_rle_t &dst, const morph_rle_t &src, morph_se_t se, void *ws,
                       hipStream_t s)
{
    const int P = src.npages, H = src.height, W = src.width;
    const long long rows = (long long)P * H;
    const BandWs L = band_ws(op, W, rows, se);
    char *w = (char *)ws;
    int *counts = (int *)w;
    int *tmp = (int *)(w + L.counts);
    int *defer = (int *)(w + L.counts + L.tmp);
    unsigned *fb = (unsigned *)(w + L.counts + L.tmp + L.defer);
    BandArgs A{};
    A.rp = src.row_ptr;
    A.runs = (const int2 *)src.runs;
    A.cap_in = src.capacity;
    A.W = W;
    A.H = H;
    A.P = P;
    A.nch = band_chains(op, se, A.ch, A.out_comp);
    const int halo = band_halo(op, se);
    A.R = std::max(1, std::min(128, kBandRowsMax - halo));
    A.nbands = (H + A.R - 1) / A.R;
    A.counts = counts;
    A.defer_n = defer;
    A.defer_rows = defer + 1;
    const long long nb = (long long)A.nbands * P;
    if (nb > 0x7fffffffLL || rows >= 0x7fffffffLL) return hipErrorInvalidValue;
    unsigned long long *tr = trace_counters();
    hipLaunchKernelGGL(clear_one_kernel, dim3(1), dim3(64), 0, s, defer);
    // count launch: reads the band's runs (with halos), writes a count per row
    trace_before(MORPH_K_RLE_BAND_COUNT, s);
    hipLaunchKernelGGL(rle_band_kernel<false>, dim3((unsigned)nb), dim3(kBT), 0, s, A);
    trace_after(MORPH_K_RLE_BAND_COUNT, s, 4.0 * (double)(rows + 1) + 4.0 * (double)rows);
    hipLaunchKernelGGL(rle_band_fallback_kernel<false>, dim3(kFallbackGroups), dim3(kBT), 0, s, A, fb, L.fb_cap,
                       L.fb_rows);
    hipError_t e = exclusive_scan(counts, (int)rows, dst.row_ptr, tmp, s);
    if (e != hipSuccess) return e;
    A.out_rp = dst.row_ptr;
    A.out_runs = (int2 *)dst.runs;
    A.cap_out = dst.capacity;
    A.trace = tr ? tr + (long long)MORPH_K_RLE_BAND * 2 * 256 * 16 : nullptr;
    // emit launch: the same rows again, the runs written at row_ptr (8 bytes
    // per run read and written come from the counters)
    trace_before(MORPH_K_RLE_BAND, s);
    hipLaunchKernelGGL(rle_band_kernel<true>, dim3((unsigned)nb), dim3(kBT), 0, s, A);
    trace_after(MORPH_K_RLE_BAND, s, 8.0 * (double)(rows + 1));
    hipLaunchKernelGGL(rle_band_fallback_kernel<true>, dim3(kFallbackGroups), dim3(kBT), 0, s, A, fb, L.fb_cap,
                       L.fb_rows);
    return hipGetLastError();
}

}  // namespace morph
