// Connected components and statistics of run-length images (section
// "Connected Component Extraction and Statistics") and run-length
// statistics (section "Other Operations").
//
// Components: every run starts as its own union-find set; every run of a
// row is united with each run of the row above that touches it (the
// intervals overlap, widened by one pixel for 8-connectivity).  The
// union links the larger root under the smaller by compare-and-swap, so
// the root of a component ends as its smallest run index: its first run in
// raster order.  The roots are counted per row; a scan of those counts
// numbers the components of each page in raster order, and every run takes
// its root's number.  All kernels give one 16-lane group to a
// row and run through the row's runs in steps of 16.
#include "common.h"

namespace morph {
namespace {

constexpr int kCcGroup = 16;
constexpr int kCcGroupsPerBlock = 256 / kCcGroup;

__device__ __forceinline__ int cc_glane() { return (int)(threadIdx.x & (kCcGroup - 1)); }

// Runs [b0, b1) of row r, offsets clamped to [0, nmax].
__device__ __forceinline__ void cc_row(const int *rp, long long r, long long nmax, int &b0, int &b1)
{
    const long long a = min((long long)max(rp[r], 0), nmax);
    b0 = (int)a;
    b1 = (int)max(a, min((long long)rp[r + 1], nmax));
}

__device__ __forceinline__ int cc_load(int *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void cc_store(int *p, int v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Root of x, halving the path on the way: parents only ever move to smaller
// indices of the same set, so a stale read still leads to the root.
__device__ __forceinline__ int cc_find(int *parent, int x)
{
    int p = cc_load(parent + x);
    while (p != x) {
        const int gp = cc_load(parent + p);
        if (gp != p) cc_store(parent + x, gp);
        x = p;
        p = gp;
    }
    return x;
}

__device__ __forceinline__ void cc_unite(int *parent, int a, int b)
{
    for (;;) {
        a = cc_find(parent, a);
        b = cc_find(parent, b);
        if (a == b) return;
        if (a < b) {
            const int t = a;
            a = b;
            b = t;
        }
        if (atomicCAS(parent + a, a, b) == a) return;   // a was still a root: linked
    }
}

// Union-find inside bands of kBandRows rows of a page, in LDS: the runs of
// a band get local parents, the runs of each row are united with the
// touching runs of the row above within the band, and every run's global
// parent is set to the first run of its band-local set.  A band with more
// runs than the LDS table holds does the same on the global parents (only
// runs of its own band are touched, which its own threads initialised).
// The rows that start a band are then joined to the row above by
// cc_merge_kernel.
constexpr int kBandRows = 32;
constexpr int kBandRuns = 4096;

__device__ __forceinline__ int lds_find(int *lp, int x)
{
    int p = __hip_atomic_load(lp + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    while (p != x) {
        x = p;
        p = __hip_atomic_load(lp + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    return x;
}

__device__ __forceinline__ void lds_unite(int *lp, int a, int b)
{
    for (;;) {
        a = lds_find(lp, a);
        b = lds_find(lp, b);
        if (a == b) return;
        if (a < b) {
            const int t = a;
            a = b;
            b = t;
        }
        if (atomicCAS(lp + a, a, b) == a) return;
    }
}

__global__ __launch_bounds__(256) void cc_band_kernel(const int *__restrict__ rp, const int2 *__restrict__ runs,
                                                      int H, int bands_per_page, long long nbands, long long nmax,
                                                      int widen, int *__restrict__ parent)
{
    __shared__ int lp[kBandRuns];
    const long long band = xcd_block();
    if (band >= nbands) return;             // whole workgroup
    const long long page = band / bands_per_page;
    const int y0 = (int)(band - page * bands_per_page) * kBandRows;
    const long long r0 = page * H + y0, r1 = page * H + min(H, y0 + kBandRows);
    const long long g0 = min((long long)max(rp[r0], 0), nmax);
    const long long g1 = max(g0, min((long long)rp[r1], nmax));
    const int n = (int)(g1 - g0);
    const bool local = n <= kBandRuns;
    for (int k = threadIdx.x; k < n; k += 256) {
        if (local) lp[k] = k; else parent[g0 + k] = (int)(g0 + k);
    }
    __syncthreads();
    for (long long r = r0 + 1 + (threadIdx.x >> 4); r < r1; r += kCcGroupsPerBlock) {
        int b0, b1, a0, a1;
        cc_row(rp, r, nmax, b0, b1);
        cc_row(rp, r - 1, nmax, a0, a1);
        if (a0 == a1) continue;
        for (int i = b0 + cc_glane(); i < b1; i += kCcGroup) {
            const int2 q = runs[i];
            int lo = a0, hi = a1;           // first run above whose end + widen passes s
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (runs[mid].y + widen > q.x) hi = mid; else lo = mid + 1;
            }
            for (int j = lo; j < a1; j++) {
                if (runs[j].x >= q.y + widen) break;
                if (local) lds_unite(lp, i - (int)g0, j - (int)g0); else cc_unite(parent, i, j);
            }
        }
    }
    __syncthreads();
    if (local)
        for (int k = threadIdx.x; k < n; k += 256) parent[g0 + k] = (int)(g0 + lds_find(lp, k));
}

__global__ __launch_bounds__(256) void cc_merge_kernel(const int *__restrict__ rp, const int2 *__restrict__ runs,
                                                       long long R, int H, long long nmax, int widen,
                                                       int *__restrict__ parent)
{
    // rows that start a band (and not a page): b-th such row of the image
    const long long b = (long long)xcd_block() * kCcGroupsPerBlock + (threadIdx.x >> 4);
    const long long per_page = (H - 1) / kBandRows;          // band starts below row 0
    if (per_page == 0 || b >= per_page * (R / H)) return;
    const long long r = (b / per_page) * H + (b % per_page + 1) * kBandRows;
    int b0, b1, a0, a1;
    cc_row(rp, r, nmax, b0, b1);
    cc_row(rp, r - 1, nmax, a0, a1);
    if (a0 == a1) return;
    for (int i = b0 + cc_glane(); i < b1; i += kCcGroup) {
        const int2 q = runs[i];
        int lo = a0, hi = a1;               // first run above whose end + widen passes s
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (runs[mid].y + widen > q.x) hi = mid; else lo = mid + 1;
        }
        for (int j = lo; j < a1; j++) {
            if (runs[j].x >= q.y + widen) break;
            cc_unite(parent, i, j);
        }
    }
}

// Counts the roots of each row (the links are final: a root is a run that
// is its own parent).
__global__ __launch_bounds__(256) void cc_roots_kernel(const int *__restrict__ rp, long long R, long long nmax,
                                                       const int *__restrict__ parent, int *__restrict__ roots)
{
    const long long r = (long long)xcd_block() * kCcGroupsPerBlock + (threadIdx.x >> 4);
    const bool live = r < R;
    int b0 = 0, b1 = 0;
    if (live) cc_row(rp, r, nmax, b0, b1);
    int n = 0;
    for (int i = b0 + cc_glane(); i < b1; i += kCcGroup) n += (parent[i] == i);
    // sum over the group
    for (int d = kCcGroup / 2; d >= 1; d >>= 1) n += __shfl_xor(n, d, kCcGroup);
    if (live && cc_glane() == 0) roots[r] = n;
}

// Number of every root within its page: the roots before its row plus
// those before it in the row, less the roots before the page's first row.
// Row 0 of each page records where the page's components begin; the last
// row records the total.
__global__ __launch_bounds__(256) void cc_rank_kernel(const int *__restrict__ rp, long long R, int H, int P,
                                                      long long nmax, const int *__restrict__ parent,
                                                      const int *__restrict__ row_base, int *__restrict__ labels,
                                                      int *__restrict__ comp_ptr)
{
    const long long r = (long long)xcd_block() * kCcGroupsPerBlock + (threadIdx.x >> 4);
    const bool live = r < R;
    int b0 = 0, b1 = 0;
    if (live) cc_row(rp, r, nmax, b0, b1);
    const int gl = cc_glane(), gbase = (int)(threadIdx.x & 63) & ~(kCcGroup - 1);
    int base = live ? row_base[r] - row_base[(r / H) * H] : 0;
    // every lane of the group takes the same number of steps (ballot below)
    for (int i0 = b0; i0 < b1; i0 += kCcGroup) {
        const int i = i0 + gl;
        const bool root = i < b1 && parent[i] == i;
        const unsigned long long m = __ballot(root);
        const unsigned gm = (unsigned)(m >> gbase) & 0xffffu;
        if (root) labels[i] = base + __popc(gm & ((1u << gl) - 1));
        base += __popc(gm);
    }
    if (live && gl == 0) {
        if (r % H == 0) comp_ptr[r / H] = row_base[r];
        if (r == R - 1) comp_ptr[P] = rp[R] > nmax ? -1 : row_base[R];   // -1: more runs than room
    }
}

// Every run that is not a root takes its root's number (the links are
// final, so the walk to the root only reads).
__global__ __launch_bounds__(256) void cc_relabel_kernel(const int *__restrict__ rp, long long R, long long nmax,
                                                         const int *__restrict__ parent, int *__restrict__ labels)
{
    const long long r = (long long)xcd_block() * kCcGroupsPerBlock + (threadIdx.x >> 4);
    if (r >= R) return;
    int b0, b1;
    cc_row(rp, r, nmax, b0, b1);
    for (int i = b0 + cc_glane(); i < b1; i += kCcGroup) {
        int root = parent[i];
        if (root == i) continue;
        for (int p = parent[root]; p != root; p = parent[root]) root = p;
        labels[i] = labels[root];
    }
}

__global__ __launch_bounds__(256) void cc_stats_init_kernel(morph_component_t *st, long long n)
{
    const long long c = (long long)blockIdx.x * 256 + threadIdx.x;
    if (c >= n) return;
    st[c] = morph_component_t{0x7fffffff, 0x7fffffff, -1, -1, 0, 0, 0};
}

// One workgroup per kStatRows rows: each run's contribution goes into an
// LDS table keyed by component (open addressing, a few probes; a run whose
// component finds no slot goes straight to the global record), and the
// table is added to the global records once at the end, so a component
// that spans many rows costs one set of global atomics per workgroup
// instead of one per run.
constexpr int kStatRows = 64;
constexpr int kStatSlots = 512;
constexpr int kStatProbes = 8;

__device__ __forceinline__ void stat_add(int *x0, int *y0, int *x1, int *y1, unsigned long long *area,
                                         unsigned long long *sx, unsigned long long *sy, int a, int b, int y)
{
    const long long len = b - a;
    atomicMin(x0, a);
    atomicMin(y0, y);
    atomicMax(x1, b);
    atomicMax(y1, y + 1);
    atomicAdd(area, (unsigned long long)len);
    atomicAdd(sx, (unsigned long long)(((long long)a + b - 1) * len / 2));
    atomicAdd(sy, (unsigned long long)((long long)y * len));
}

__global__ __launch_bounds__(256) void cc_stats_kernel(const int *__restrict__ rp, const int2 *__restrict__ runs,
                                                       long long R, int H, long long nmax,
                                                       const int *__restrict__ labels,
                                                       const int *__restrict__ comp_ptr, morph_component_t *st,
                                                       long long ncap)
{
    __shared__ long long key[kStatSlots];
    __shared__ int bx0[kStatSlots], by0[kStatSlots], bx1[kStatSlots], by1[kStatSlots];
    __shared__ unsigned long long bar[kStatSlots], bsx[kStatSlots], bsy[kStatSlots];
    for (int k = threadIdx.x; k < kStatSlots; k += 256) {
        key[k] = -1;
        bx0[k] = by0[k] = 0x7fffffff;
        bx1[k] = by1[k] = -1;
        bar[k] = bsx[k] = bsy[k] = 0;
    }
    __syncthreads();
    const long long r0 = (long long)xcd_block() * kStatRows;
    for (long long r = r0 + (threadIdx.x >> 4); r < min(R, r0 + kStatRows); r += kCcGroupsPerBlock) {
        int b0, b1;
        cc_row(rp, r, nmax, b0, b1);
        const int y = (int)(r % H);
        const long long first = comp_ptr[r / H];
        for (int i = b0 + cc_glane(); i < b1; i += kCcGroup) {
            const int2 q = runs[i];
            const long long c = first + labels[i];
            if (c < 0 || c >= ncap) continue;
            int slot = -1;
            int h = (int)((unsigned long long)(c * 0x9E3779B97F4A7C15ull) >> 55) & (kStatSlots - 1);
            for (int t = 0; t < kStatProbes; t++) {
                const unsigned long long prev = atomicCAS((unsigned long long *)&key[h], ~0ull,
                                                          (unsigned long long)c);
                if (prev == ~0ull || prev == (unsigned long long)c) {
                    slot = h;
                    break;
                }
                h = (h + 1) & (kStatSlots - 1);
            }
            if (slot >= 0) {
                stat_add(&bx0[slot], &by0[slot], &bx1[slot], &by1[slot], &bar[slot], &bsx[slot], &bsy[slot],
                         q.x, q.y, y);
            } else {
                morph_component_t *g = st + c;
                stat_add(&g->x0, &g->y0, &g->x1, &g->y1, (unsigned long long *)&g->area,
                         (unsigned long long *)&g->sum_x, (unsigned long long *)&g->sum_y, q.x, q.y, y);
            }
        }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < kStatSlots; k += 256) {
        const long long c = key[k];
        if (c < 0) continue;
        morph_component_t *g = st + c;
        atomicMin(&g->x0, bx0[k]);
        atomicMin(&g->y0, by0[k]);
        atomicMax(&g->x1, bx1[k]);
        atomicMax(&g->y1, by1[k]);
        atomicAdd((unsigned long long *)&g->area, bar[k]);
        atomicAdd((unsigned long long *)&g->sum_x, bsx[k]);
        atomicAdd((unsigned long long *)&g->sum_y, bsy[k]);
    }
}

// ------------------------------------------------------ run-length statistics
// One workgroup per range of kHistRows rows of one page; its 16-lane groups
// take rows in turn and count run and gap lengths in LDS histograms (when
// 2 (W + 1) counters fit), which are added to the page's histograms at the
// end.
constexpr int kHistRows = 256;
constexpr int kHistLdsBins = 8192;      // counters per histogram kept in LDS at most

__global__ __launch_bounds__(256) void run_hist_kernel(const int *__restrict__ rp, const int2 *__restrict__ runs,
                                                       int H, int W, long long nmax, int ranges,
                                                       int *__restrict__ black, int *__restrict__ white)
{
    extern __shared__ int hist_lds[];       // 2 (W + 1) counters when local
    const int page = (int)(blockIdx.x / ranges), range = (int)(blockIdx.x % ranges);
    const int nb = W + 1;
    const bool local = nb <= kHistLdsBins;
    int *lb = hist_lds, *lw = hist_lds + nb;
    int *gb = black + (long long)page * nb, *gw = white + (long long)page * nb;
    if (local)
        for (int b = threadIdx.x; b < nb; b += 256) {
            lb[b] = 0;
            lw[b] = 0;
        }
    __syncthreads();
    const int y1 = min(H, (range + 1) * kHistRows);
    for (int y = range * kHistRows + (int)(threadIdx.x >> 4); y < y1; y += kCcGroupsPerBlock) {
        int b0, b1;
        cc_row(rp, (long long)page * H + y, nmax, b0, b1);
        for (int i = b0 + cc_glane(); i < b1; i += kCcGroup) {
            const int2 q = runs[i];
            const int len = min(max(q.y - q.x, 0), W);
            if (local) atomicAdd(&lb[len], 1); else atomicAdd(&gb[len], 1);
            if (i > b0) {
                const int gap = min(max(q.x - runs[i - 1].y, 0), W);
                if (local) atomicAdd(&lw[gap], 1); else atomicAdd(&gw[gap], 1);
            }
        }
    }
    __syncthreads();
    if (local)
        for (int b = threadIdx.x; b < nb; b += 256) {
            if (lb[b]) atomicAdd(&gb[b], lb[b]);
            if (lw[b]) atomicAdd(&gw[b], lw[b]);
        }
}

__global__ __launch_bounds__(256) void zero_ints_kernel(int *p, long long n)
{
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = 0;
}

// Sum of the histograms of all rows per bin: a grid over (bin chunk, row
// chunk), each thread adding up to kSumRows rows of one bin.
constexpr int kSumRows = 16;

__global__ __launch_bounds__(256) void hist_sum_kernel(const int *__restrict__ hist, int nrows, int nbins,
                                                       int *__restrict__ sum)
{
    const int b = (int)(blockIdx.x * 256 + threadIdx.x);
    if (b >= nbins) return;
    const int p0 = (int)blockIdx.y * kSumRows, p1 = min(nrows, p0 + kSumRows);
    int v = 0;
    for (int p = p0; p < p1; p++) v += hist[(long long)p * nbins + b];
    if (v) atomicAdd(sum + b, v);
}

// One workgroup over a single histogram (the sum over rows): its total,
// then the first bin at which the running count reaches num/den of it.
__global__ __launch_bounds__(256) void percentile_kernel(const int *__restrict__ hist, int nrows, int nbins,
                                                         long long num, long long den, int *out)
{
    __shared__ long long part[256];
    __shared__ long long carry_s;
    __shared__ int found;
    const int t = (int)threadIdx.x;
    long long tot = 0;
    for (int b = t; b < nbins; b += 256)
        for (int p = 0; p < nrows; p++) tot += hist[(long long)p * nbins + b];
    part[t] = tot;
    __syncthreads();
    for (int d = 128; d >= 1; d >>= 1) {
        if (t < d) part[t] += part[t + d];
        __syncthreads();
    }
    const long long total = part[0];
    __syncthreads();
    if (t == 0) {
        carry_s = 0;
        found = total == 0 ? 0 : nbins - 1;
    }
    __syncthreads();
    if (total == 0) {
        if (t == 0) out[0] = 0;
        return;
    }
    for (int c0 = 0; c0 < nbins; c0 += 256) {
        const int b = c0 + t;
        long long v = 0;
        if (b < nbins)
            for (int p = 0; p < nrows; p++) v += hist[(long long)p * nbins + b];
        part[t] = v;
        __syncthreads();
        for (int d = 1; d < 256; d <<= 1) {             // inclusive scan of the chunk
            const long long add = t >= d ? part[t - d] : 0;
            __syncthreads();
            part[t] += add;
            __syncthreads();
        }
        const long long cum = carry_s + part[t];
        const bool hit = b < nbins && cum * den >= total * num;
        const bool prev = t > 0 ? (carry_s + part[t - 1]) * den >= total * num : carry_s * den >= total * num;
        if (hit && !prev) atomicMin(&found, b);
        __syncthreads();
        if (t == 255) carry_s += part[255];
        __syncthreads();
        if (carry_s * den >= total * num) break;
    }
    if (t == 0) out[0] = found;
}

unsigned cc_blocks(long long rows) { return (unsigned)((rows + kCcGroupsPerBlock - 1) / kCcGroupsPerBlock); }

}  // namespace

// ------------------------------------------------------------------ host
size_t cc_workspace(long long R, long long nruns)
{
    const auto r256 = [](size_t b) { return (b + 255) & ~(size_t)255; };
    return r256((size_t)nruns * 4) + r256((size_t)R * 4) + r256((size_t)(R + 1) * 4) + scan_workspace(R);
}

hipError_t cc_label(const morph_rle_t &src, int connectivity, int *labels, long long nmax, int *comp_ptr,
                    void *ws, hipStream_t s)
{
    const long long R = (long long)src.height * src.npages;
    const auto r256 = [](size_t b) { return (b + 255) & ~(size_t)255; };
    char *w = (char *)ws;
    int *parent = (int *)w;
    int *roots = (int *)(w + r256((size_t)nmax * 4));
    int *row_base = (int *)((char *)roots + r256((size_t)R * 4));
    int *tmp = (int *)((char *)row_base + r256((size_t)(R + 1) * 4));
    const unsigned g = cc_blocks(R);
    const int2 *runs = reinterpret_cast<const int2 *>(src.runs);
    trace_before(MORPH_K_COMPONENTS, s);
    const int bpp = (src.height + kBandRows - 1) / kBandRows;
    const long long nbands = (long long)bpp * src.npages;
    const int widen = connectivity == 8 ? 1 : 0;
    hipLaunchKernelGGL(cc_band_kernel, dim3((unsigned)nbands), dim3(256), 0, s, src.row_ptr, runs, src.height, bpp,
                       nbands, nmax, widen, parent);
    const long long starts = (long long)((src.height - 1) / kBandRows) * src.npages;
    if (starts > 0)
        hipLaunchKernelGGL(cc_merge_kernel, dim3(cc_blocks(starts)), dim3(256), 0, s, src.row_ptr, runs, R,
                           src.height, nmax, widen, parent);
    hipLaunchKernelGGL(cc_roots_kernel, dim3(g), dim3(256), 0, s, src.row_ptr, R, nmax, parent, roots);
    hipError_t e = exclusive_scan(roots, (int)R, row_base, tmp, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(cc_rank_kernel, dim3(g), dim3(256), 0, s, src.row_ptr, R, src.height, src.npages, nmax,
                       parent, row_base, labels, comp_ptr);
    hipLaunchKernelGGL(cc_relabel_kernel, dim3(g), dim3(256), 0, s, src.row_ptr, R, nmax, parent, labels);
    trace_after(MORPH_K_COMPONENTS, s, 4.0 * (R + 1) + 4.0 * (src.npages + 1));
    return hipGetLastError();
}

hipError_t cc_stats(const morph_rle_t &src, const int *labels, long long nmax, const int *comp_ptr,
                    morph_component_t *st, long long ncap, hipStream_t s)
{
    const long long R = (long long)src.height * src.npages;
    trace_before(MORPH_K_COMPONENT_STATS, s);
    if (ncap > 0)
        hipLaunchKernelGGL(cc_stats_init_kernel, dim3((unsigned)((ncap + 255) / 256)), dim3(256), 0, s, st, ncap);
    hipLaunchKernelGGL(cc_stats_kernel, dim3((unsigned)((R + kStatRows - 1) / kStatRows)), dim3(256), 0, s,
                       src.row_ptr,
                       reinterpret_cast<const int2 *>(src.runs), R, src.height, nmax, labels, comp_ptr, st, ncap);
    trace_after(MORPH_K_COMPONENT_STATS, s, 4.0 * (R + 1) + (double)ncap * sizeof(morph_component_t));
    return hipGetLastError();
}

hipError_t run_histograms(const morph_rle_t &src, int *black, int *white, hipStream_t s)
{
    const long long n = (long long)src.npages * (src.width + 1);
    const int ranges = (src.height + kHistRows - 1) / kHistRows;
    trace_before(MORPH_K_HISTOGRAM, s);
    hipLaunchKernelGGL(zero_ints_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, black, n);
    hipLaunchKernelGGL(zero_ints_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, white, n);
    const size_t lds = (src.width + 1 <= kHistLdsBins) ? 2 * (size_t)(src.width + 1) * sizeof(int) : 0;
    hipLaunchKernelGGL(run_hist_kernel, dim3((unsigned)((long long)src.npages * ranges)), dim3(256), lds, s,
                       src.row_ptr, reinterpret_cast<const int2 *>(src.runs), src.height, src.width,
                       (long long)src.capacity, ranges, black, white);
    trace_after(MORPH_K_HISTOGRAM, s, 4.0 * ((double)src.height * src.npages + 1) + 8.0 * n);
    return hipGetLastError();
}

size_t percentile_workspace(int nbins) { return ((size_t)nbins * 4 + 255) & ~(size_t)255; }

hipError_t histogram_percentile(const int *hist, int nrows, int nbins, int num, int den, int *out, void *ws,
                                hipStream_t s)
{
    int *sum = (int *)ws;
    hipLaunchKernelGGL(zero_ints_kernel, dim3((unsigned)((nbins + 255) / 256)), dim3(256), 0, s, sum,
                       (long long)nbins);
    hipLaunchKernelGGL(hist_sum_kernel, dim3((unsigned)((nbins + 255) / 256), (unsigned)((nrows + kSumRows - 1) / kSumRows)),
                       dim3(256), 0, s, hist, nrows, nbins, sum);
    hipLaunchKernelGGL(percentile_kernel, dim3(1), dim3(256), 0, s, sum, 1, nbins, (long long)num,
                       (long long)den, out);
    return hipGetLastError();
}

}  // namespace morph
