// Packed-bitmap rectangle morphology on gfx950: one fused band kernel.
//
// The method (paper, sections "Efficient Binary Decompositions" and "2D
// Morphological Operators for Rectangular Masks"): a rectangle is separable,
// so an operation is a row pass followed by a column pass, and each pass
// covers a line of n pixels by logarithmic decomposition: E_1 = A,
// E_2k(p) = E_k(p) AND E_k(p+k) while 2k <= n, one more step with offset
// n - m (m the largest power of two <= n), then a shift that puts the origin
// in place.  Only erosion is implemented in the kernel; dilation, opening
// and closing are erosions of complements (dilation_B(A) = NOT
// erosion_B^(NOT A) with B^ the reflected element, and the outside value 0
// of dilation becomes the outside value 1 of erosion under the complement).
//
// One workgroup computes one tile: TR output rows x SW words of one page.
// It stages the rows the tile depends on (TR + sum(h-1) of them, plus one
// halo word per side and stage) in LDS with the border already filled, runs
// the row pass in registers on 4-word groups with cross-word funnel shifts,
// then the column pass with each thread holding a run of rows of one word
// column in registers and exchanging only the rows its neighbour needs
// through LDS.  With two stages (opening, closing) the intermediate never
// leaves LDS: it is complemented, clipped to the page and fed to the second
// stage.  Global memory is read once and written once per tile (halo rows
// and words are re-read from cache by the neighbouring tile).
#include "common.h"

#include <algorithm>

namespace morph {

namespace {

constexpr uint64_t kOnes = ~0ull;
constexpr int WPT = kWordsPerItem;
constexpr int CM = kChunkMax;

// Low 64 bits of the 128-bit value (hi:lo) shifted right by s, 1 <= s <= 63.
__device__ __forceinline__ uint64_t funnel_r(uint64_t hi, uint64_t lo, int s)
{
    const uint32_t l0 = (uint32_t)lo, l1 = (uint32_t)(lo >> 32);
    const uint32_t h0 = (uint32_t)hi, h1 = (uint32_t)(hi >> 32);
    uint32_t r0, r1;
    if (s < 32) {
        r0 = __builtin_amdgcn_alignbit(l1, l0, (uint32_t)s);
        r1 = __builtin_amdgcn_alignbit(h0, l1, (uint32_t)s);
    } else {
        r0 = __builtin_amdgcn_alignbit(h0, l1, (uint32_t)(s - 32));
        r1 = __builtin_amdgcn_alignbit(h1, h0, (uint32_t)(s - 32));
    }
    return ((uint64_t)r1 << 32) | r0;
}

// One doubling step along a row: E(p) &= E(p + K), over a window of
// WPT + 2 consecutive words (bit p of word i is pixel 64*i + p).  The last
// word's high bits would need the word after it; they are never used.
template <int K>
__device__ __forceinline__ void row_step(uint64_t (&X)[WPT + 2])
{
#pragma unroll
    for (int i = 0; i < WPT + 1; i++) {
        const uint64_t nb = (K == 64) ? X[i + 1] : funnel_r(X[i + 1], X[i], K);
        X[i] &= nb;
    }
    if (K < 64) X[WPT + 1] &= (X[WPT + 1] >> (K & 63)) | (kOnes << ((64 - K) & 63));
}

__device__ __forceinline__ void row_step_rt(uint64_t (&X)[WPT + 2], int s)
{
#pragma unroll
    for (int i = 0; i < WPT + 1; i++) X[i] &= funnel_r(X[i + 1], X[i], s);
    X[WPT + 1] &= (X[WPT + 1] >> s) | (kOnes << (64 - s));
}

// Row pass for one group: X[0] is the word left of the group, X[1..WPT] the
// group, X[WPT+1] the word right of it.  out(x) = AND of A(x-cx .. x-cx+w-1)
// for the WPT words of the group.  Needs cx <= 64 and w-1-cx <= 64.
__device__ __forceinline__ void row_pass_group(uint64_t (&X)[WPT + 2], int w, int cx,
                                               uint64_t (&out)[WPT])
{
    int m = 1;
    if (w >= 2)   { row_step<1>(X);  m = 2; }
    if (w >= 4)   { row_step<2>(X);  m = 4; }
    if (w >= 8)   { row_step<4>(X);  m = 8; }
    if (w >= 16)  { row_step<8>(X);  m = 16; }
    if (w >= 32)  { row_step<16>(X); m = 32; }
    if (w >= 64)  { row_step<32>(X); m = 64; }
    if (w >= 128) { row_step<64>(X); m = 128; }
    if (w > m) row_step_rt(X, w - m);
    // origin: out(x) = E_w(x - cx)
#pragma unroll
    for (int i = 0; i < WPT; i++)
        out[i] = (cx == 0) ? X[i + 1] : (cx == 64 ? X[i] : funnel_r(X[i + 1], X[i], 64 - cx));
}

// Column doubling step with a compile-time offset K < CM: partners inside
// the thread's own run of rows come from registers, the others from LDS,
// where every thread first publishes the rows its upper neighbour needs.
template <int K>
__device__ __forceinline__ void col_step(uint64_t *lds, uint64_t (&reg)[CM], int TW, int NRs,
                                         int col, int a, int C, bool active)
{
    __syncthreads();
    if (active) {
#pragma unroll
        for (int i = 0; i < (K < CM ? K : CM); i++)
            if (i < C && a + i < NRs) lds[(a + i) * TW + col] = reg[i];
    }
    __syncthreads();
    if (active) {
#pragma unroll
        for (int i = 0; i < CM; i++) {
            if (i < C) {
                uint64_t p;
                if (i + K < C) {
                    p = reg[(i + K < CM) ? i + K : CM - 1];
                } else {
                    const int rr = a + i + K;
                    p = rr < NRs ? lds[rr * TW + col] : kOnes;
                }
                reg[i] &= p;
            }
        }
    }
}

// Column step with a run-time offset: every partner comes from LDS.
__device__ __forceinline__ void col_step_lds(uint64_t *lds, uint64_t (&reg)[CM], int TW, int NRs,
                                             int col, int a, int C, bool active, int K)
{
    __syncthreads();
    if (active) {
#pragma unroll
        for (int i = 0; i < CM; i++)
            if (i < C && a + i < NRs) lds[(a + i) * TW + col] = reg[i];
    }
    __syncthreads();
    if (active) {
#pragma unroll
        for (int i = 0; i < CM; i++) {
            if (i < C) {
                const int rr = a + i + K;
                reg[i] &= rr < NRs ? lds[rr * TW + col] : kOnes;
            }
        }
    }
}

__device__ __forceinline__ void rect_tile(const RectPage &P, int page, int band, int strip, uint64_t *lds)
{
    const int tid = threadIdx.x;
    const uint64_t *src = P.src + (long long)page * P.src_page_words;
    uint64_t *dst = P.dst + (long long)page * P.dst_page_words;
    const int nst = P.nst;
    const int y0 = band * P.TR;
    const int TRv = min(P.TR, P.H - y0);
    const int j0 = strip * P.SW;
    const int SWv = min(P.SW, P.nw - j0);
    const int TW = SWv + 2 * nst;
    int hsum = P.st[0].h - 1, top = P.st[0].cy;
    if (nst == 2) { hsum += P.st[1].h - 1; top += P.st[1].cy; }
    int NRs = TRv + hsum;           // rows held in LDS for the current stage
    int gy0 = y0 - top;             // page row of LDS row 0
    const int gj0 = j0 - nst;       // page word of LDS column 0

    // ---- stage the input rows; outside the page every pixel is 1
    {
        const int total = NRs * TW;
        int r = tid / TW, c = tid - (tid / TW) * TW;
        const int dr = kThreads / TW, dc = kThreads - (kThreads / TW) * TW;
        for (int q = tid; q < total; q += kThreads) {
            const int gy = gy0 + r, gj = gj0 + c;
            uint64_t v = kOnes;
            if (gy >= 0 && gy < P.H && gj >= 0 && gj < P.nw) {
                v = src[(long long)gy * P.sstride + gj];
                if (P.in_c) v = ~v;
                if (gj == P.nw - 1) v |= ~P.padmask;
            }
            lds[q] = v;
            r += dr;
            c += dc;
            if (c >= TW) { c -= TW; r++; }
        }
    }
    __syncthreads();

    for (int s = 0; s < nst; s++) {
        const Stage S = (s == 0) ? P.st[0] : P.st[1];
        const int c_lo = 1 + s, c_hi = TW - 1 - s;

        // ---- row pass, in place on columns [c_lo, c_hi)
        if (S.w > 1) {
            const int G = (c_hi - c_lo + WPT - 1) / WPT;
            const int items = NRs * G;
            const int dr = kThreads / G, dg = kThreads - (kThreads / G) * G;
            uint64_t res[kItemsMax][WPT];
            int r = tid / G, g = tid - (tid / G) * G;
#pragma unroll
            for (int k = 0; k < kItemsMax; k++) {
                if (tid + k * kThreads < items) {
                    const int c0 = c_lo + g * WPT;
                    uint64_t X[WPT + 2];
#pragma unroll
                    for (int i = 0; i < WPT + 2; i++) {
                        const int c = c0 - 1 + i;
                        X[i] = c < TW ? lds[r * TW + c] : kOnes;
                    }
                    row_pass_group(X, S.w, S.cx, res[k]);
                }
                r += dr;
                g += dg;
                if (g >= G) { g -= G; r++; }
            }
            __syncthreads();
            r = tid / G;
            g = tid - (tid / G) * G;
#pragma unroll
            for (int k = 0; k < kItemsMax; k++) {
                if (tid + k * kThreads < items) {
                    const int c0 = c_lo + g * WPT;
#pragma unroll
                    for (int i = 0; i < WPT; i++)
                        if (c0 + i < c_hi) lds[r * TW + c0 + i] = res[k][i];
                }
                r += dr;
                g += dg;
                if (g >= G) { g -= G; r++; }
            }
            __syncthreads();
        }

        // ---- column pass on columns [c_lo, c_hi)
        const int ncols = c_hi - c_lo;
        const int chunks = kThreads / ncols;
        const int C = (NRs + chunks - 1) / chunks;
        const int chunk = tid / ncols;
        const int col = c_lo + (tid - chunk * ncols);
        const bool active = chunk < chunks;
        const int a = chunk * C;
        uint64_t reg[CM];
#pragma unroll
        for (int i = 0; i < CM; i++)
            reg[i] = (active && i < C && a + i < NRs) ? lds[(a + i) * TW + col] : kOnes;

        const int h = S.h;
        int m = 1;
        if (h >= 2)  { col_step<1>(lds, reg, TW, NRs, col, a, C, active);  m = 2; }
        if (h >= 4)  { col_step<2>(lds, reg, TW, NRs, col, a, C, active);  m = 4; }
        if (h >= 8)  { col_step<4>(lds, reg, TW, NRs, col, a, C, active);  m = 8; }
        if (h >= 16) { col_step<8>(lds, reg, TW, NRs, col, a, C, active);  m = 16; }
        if (h >= 32) { col_step<16>(lds, reg, TW, NRs, col, a, C, active); m = 32; }
        while (2 * m <= h) {
            col_step_lds(lds, reg, TW, NRs, col, a, C, active, m);
            m *= 2;
        }
        if (h > m) col_step_lds(lds, reg, TW, NRs, col, a, C, active, h - m);

        // reg[i] now holds the erosion of row a+i of this stage's output
        const int NRo = NRs - (h - 1);
        const int gyo = gy0 + S.cy;           // page row of output row 0
        if (s + 1 < nst) {
            // intermediate: (optionally complemented), clipped to the page,
            // outside = 1 for the next erosion
            __syncthreads();
            if (active) {
#pragma unroll
                for (int i = 0; i < CM; i++) {
                    const int r = a + i;
                    if (i < C && r < NRo) {
                        const int gy = gyo + r, gj = gj0 + col;
                        uint64_t v = P.mid_c ? ~reg[i] : reg[i];
                        if (gy < 0 || gy >= P.H || gj < 0 || gj >= P.nw) v = kOnes;
                        else if (gj == P.nw - 1) v |= ~P.padmask;
                        lds[r * TW + col] = v;
                    }
                }
            }
            __syncthreads();
            NRs = NRo;
            gy0 = gyo;
        } else if (active) {
            const int gj = gj0 + col;
#pragma unroll
            for (int i = 0; i < CM; i++) {
                const int r = a + i;
                if (i < C && r < NRo) {
                    uint64_t v = P.out_c ? ~reg[i] : reg[i];
                    if (gj == P.nw - 1) v &= P.padmask;
                    dst[(long long)(gyo + r) * P.dstride + gj] = v;
                }
            }
        }
    }
}

// Tiles of a launch are numbered band-major; hand consecutive tiles to the
// same XCD (workgroups are dealt round-robin over the 8 XCDs) so a tile and
// its neighbour share halo rows in one L2.
__device__ __forceinline__ int xcd_tile(int b, int T)
{
    const int q = T >> 3, rem = T & 7;
    const int x = b & 7, k = b >> 3;
    return x * q + min(x, rem) + k;
}

__global__ __launch_bounds__(kThreads) void rect_kernel(RectPage P)
{
    __shared__ uint64_t lds[kLdsWords];
    const int T = P.nbands * P.nstrips;
    const int t = xcd_tile((int)blockIdx.x, T);
    const int band = t / P.nstrips;
    rect_tile(P, (int)blockIdx.y, band, t - band * P.nstrips, lds);
}

__global__ __launch_bounds__(kThreads) void rect_batch_kernel(const RectPage *__restrict__ pages,
                                                             const TileRef *__restrict__ tiles,
                                                             int ntiles, int *queue)
{
    __shared__ uint64_t lds[kLdsWords];
    __shared__ int next;
    for (;;) {
        if (threadIdx.x == 0) next = atomicAdd(queue, 1);
        __syncthreads();
        const int t = next;
        __syncthreads();
        if (t >= ntiles) break;                 // every wave sees the same t
        const TileRef tr = tiles[t];
        const RectPage P = pages[tr.page];
        rect_tile(P, 0, tr.band, tr.strip, lds);
        __syncthreads();
    }
}

__global__ void reset_counter_kernel(int *q)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *q = 0;
}

int cached_cu_count = 0;

}  // namespace

int device_cu_count()
{
    if (cached_cu_count == 0) {
        int dev = 0, n = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && n > 0)
            cached_cu_count = n;
        else
            cached_cu_count = 256;
    }
    return cached_cu_count;
}

// Largest number of LDS rows (input rows of stage 0) a tile of width TW can
// hold for page p, or 0 if none.
static int max_rows(const RectPage &p, int TW)
{
    int nr = kLdsWords / TW;
    int drop = 0;                   // rows lost before stage s
    for (int s = 0; s < p.nst; s++) {
        const int ncols = TW - 2 - 2 * s;
        if (ncols < 1) return 0;
        const int chunks = kThreads / ncols;
        if (chunks < 1) return 0;
        nr = std::min(nr, chunks * kChunkMax + drop);
        if (p.st[s].w > 1) {
            const int G = (ncols + WPT - 1) / WPT;
            nr = std::min(nr, (kThreads * kItemsMax) / G + drop);
        }
        drop += p.st[s].h - 1;
    }
    return nr;
}

bool plan_tiles(RectPage &p, int tile_rows, int strip_words, int npages)
{
    for (int s = 0; s < p.nst; s++) {
        const Stage &S = p.st[s];
        if (S.w < 1 || S.h < 1 || S.cx < 0 || S.cy < 0 || S.cx >= S.w || S.cy >= S.h) return false;
        if (S.cx > kReachMax || S.w - 1 - S.cx > kReachMax) return false;
    }
    int hsum = 0;
    for (int s = 0; s < p.nst; s++) hsum += p.st[s].h - 1;
    int SW;
    if (strip_words > 0) {
        SW = std::min(strip_words, p.nw);
    } else {
        const int ns = (p.nw + kStripMax - 1) / kStripMax;
        SW = (p.nw + ns - 1) / ns;
    }
    int trmax = 0;
    while (SW >= 1) {
        trmax = max_rows(p, SW + 2 * p.nst) - hsum;
        if (trmax >= 1) break;
        if (SW == 1) return false;
        SW = (SW + 1) / 2;
    }
    const int nstrips = (p.nw + SW - 1) / SW;
    int TR;
    if (tile_rows > 0) {
        TR = std::min(tile_rows, trmax);
    } else {
        // enough tiles to give every CU two workgroups, without letting the
        // halo rows dominate
        const long long want = 2LL * device_cu_count();
        const long long bands = std::max<long long>(1, want / ((long long)nstrips * std::max(1, npages)));
        const int tr_par = (int)((p.H + bands - 1) / bands);
        const int floor_rows = std::min(trmax, std::max(16, 2 * hsum));
        TR = std::max(tr_par, floor_rows);
        TR = std::min(TR, trmax);
    }
    TR = std::max(1, std::min(TR, p.H));
    p.TR = TR;
    p.SW = SW;
    p.nbands = (p.H + TR - 1) / TR;
    p.nstrips = nstrips;
    return true;
}

// Re-checks, before any launch, that the tile shape fits what rect_tile
// assumes: the LDS array, the per-thread register runs of the column pass
// and the row-pass items a thread holds across a barrier.
bool tile_fits(const RectPage &p)
{
    if (p.nst < 1 || p.nst > 2 || p.TR < 1 || p.SW < 1 || p.nw < 1 || p.H < 1) return false;
    if (p.nbands != (p.H + p.TR - 1) / p.TR || p.nstrips != (p.nw + p.SW - 1) / p.SW) return false;
    int hsum = 0;
    for (int s = 0; s < p.nst; s++) {
        const Stage &S = p.st[s];
        if (S.w < 1 || S.h < 1 || S.cx < 0 || S.cx >= S.w || S.cy < 0 || S.cy >= S.h) return false;
        if (S.cx > kReachMax || S.w - 1 - S.cx > kReachMax) return false;
        hsum += S.h - 1;
    }
    const int TW = p.SW + 2 * p.nst;
    int NRs = p.TR + hsum;
    if ((long long)NRs * TW > kLdsWords) return false;
    for (int s = 0; s < p.nst; s++) {
        const int ncols = TW - 2 - 2 * s;
        const int chunks = kThreads / ncols;
        if (ncols < 1 || chunks < 1 || (NRs + chunks - 1) / chunks > kChunkMax) return false;
        if (p.st[s].w > 1 && (long long)NRs * ((ncols + WPT - 1) / WPT) > (long long)kThreads * kItemsMax)
            return false;
        NRs -= p.st[s].h - 1;
    }
    return true;
}

hipError_t launch_rect(const RectPage &p, int npages, hipStream_t stream)
{
    const long long T = (long long)p.nbands * p.nstrips;
    if (T <= 0 || npages <= 0) return hipSuccess;
    if (!tile_fits(p) || T > 0x7fffffffLL || npages > 65535) return hipErrorInvalidValue;
    dim3 grid((unsigned)T, (unsigned)npages);
    hipLaunchKernelGGL(rect_kernel, grid, dim3(kThreads), 0, stream, p);
    return hipGetLastError();
}

hipError_t launch_rect_batch(const RectPage *pages_dev, const TileRef *tiles_dev, int ntiles,
                             int *queue_dev, int nblocks, hipStream_t stream)
{
    hipLaunchKernelGGL(rect_batch_kernel, dim3(nblocks), dim3(kThreads), 0, stream, pages_dev,
                       tiles_dev, ntiles, queue_dev);
    return hipGetLastError();
}

hipError_t launch_reset_counter(int *queue_dev, hipStream_t stream)
{
    hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(64), 0, stream, queue_dev);
    return hipGetLastError();
}

}  // namespace morph
