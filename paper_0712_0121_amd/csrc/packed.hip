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


// Workgroup barrier that orders LDS only: global loads and stores in flight
// stay in flight across it.
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

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
    if (cx == 0) {
#pragma unroll
        for (int i = 0; i < WPT; i++) out[i] = X[i + 1];
    } else if (cx == 64) {
#pragma unroll
        for (int i = 0; i < WPT; i++) out[i] = X[i];
    } else {
        const int sh = 64 - cx;
#pragma unroll
        for (int i = 0; i < WPT; i++) out[i] = funnel_r(X[i + 1], X[i], sh);
    }
}

// Loads the WPT+2 words c0-1 .. c0+WPT of an LDS row (two words per load
// when the first is at an even index).
__device__ __forceinline__ void load_group(const uint64_t *row, int c0, uint64_t (&X)[WPT + 2])
{
    if (((c0 - 1) & 1) == 0) {
        const ulonglong2 *q = reinterpret_cast<const ulonglong2 *>(row + c0 - 1);
#pragma unroll
        for (int i = 0; i < (WPT + 2) / 2; i++) {
            const ulonglong2 v = q[i];
            X[2 * i] = v.x;
            X[2 * i + 1] = v.y;
        }
    } else {
#pragma unroll
        for (int i = 0; i < WPT + 2; i++) X[i] = row[c0 - 1 + i];
    }
}

// Column doubling step with a compile-time offset K < CM: partners inside
// the thread's own run of CM rows come from registers, the others from LDS,
// where every thread first publishes the K rows its upper neighbour needs.
// A stage of h rows keeps only the output rows whose window of h rows lies
// below its input rows, and every partner of such a row (at most h - 1
// rows below it) lies there too.  Partner rows at or past `rows` (the rows
// the tile allocates in LDS) therefore feed only rows that are dropped:
// they are read at the last allocated row, which keeps the access in bounds
// without a select.  The partner's word index advances by the pitch, with
// no multiply per row.
template <int K>
__device__ __forceinline__ void col_step(uint64_t *lds, uint64_t (&reg)[CM], int TWp, int rows,
                                         int col, int a, bool active)
{
    lds_barrier();
    if (active) {
#pragma unroll
        for (int i = 0; i < K; i++) lds[(a + i) * TWp + col] = reg[i];
    }
    lds_barrier();
    const int last = (rows - 1) * TWp + col;
    int idx = (a + CM) * TWp + col;         // partner of row CM - K: row a + CM
#pragma unroll
    for (int i = 0; i < CM; i++) {
        uint64_t p;
        if (i + K < CM) {
            p = reg[(i + K < CM) ? i + K : CM - 1];
        } else {
            p = lds[min(idx, last)];
            idx += TWp;
        }
        reg[i] &= p;
    }
}

// Column step with a run-time offset: every partner comes from LDS.
__device__ __forceinline__ void col_step_lds(uint64_t *lds, uint64_t (&reg)[CM], int TWp, int rows,
                                             int col, int a, bool active, int K)
{
    lds_barrier();
    if (active) {
#pragma unroll
        for (int i = 0; i < CM; i++) lds[(a + i) * TWp + col] = reg[i];
    }
    lds_barrier();
    const int last = (rows - 1) * TWp + col;
    int idx = (a + K) * TWp + col;
#pragma unroll
    for (int i = 0; i < CM; i++) {
        reg[i] &= lds[min(idx, last)];
        idx += TWp;
    }
}

// Geometry of one tile: TR output rows x SW words of one page, plus the rows
// and words it depends on.
// LDS pitch (words) of a tile row TW words wide: even, for the 16-byte row
// reads of the row pass, and for two stages 2 mod 4, so that the first
// stage's write-back of 4-word groups (whose starts lie 32 bytes apart within
// a row) spreads over twice as many banks across rows.
__host__ __device__ __forceinline__ int tile_pitch(int TW, int nst)
{
    const int p = TW + (TW & 1);
    return (nst == 2 && (p & 3) == 0) ? p + 2 : p;
}

struct Tile {
    const uint64_t *src;
    uint64_t *dst;
    int y0, TRv, j0, SWv;
    int TW, TWp;            // LDS row width and pitch (pitch even)
    int NR;                 // input rows of the first stage
    int gy0, gj0;           // page row / word of LDS row 0 / column 0
};

__device__ __forceinline__ Tile make_tile(const RectPage &P, int page, int band, int strip)
{
    Tile T;
    T.src = P.src + (long long)page * P.src_page_words;
    T.dst = P.dst + (long long)page * P.dst_page_words;
    T.y0 = band * P.TR;
    T.TRv = min(P.TR, P.H - T.y0);
    T.j0 = strip * P.SW;
    T.SWv = min(P.SW, P.nw - T.j0);
    T.TW = T.SWv + 2 * P.nst;
    T.TWp = tile_pitch(T.TW, P.nst);
    int hsum = P.st[0].h - 1, top = P.st[0].cy;
    if (P.nst == 2) { hsum += P.st[1].h - 1; top += P.st[1].cy; }
    T.NR = T.TRv + hsum;
    T.gy0 = T.y0 - top;
    T.gj0 = T.j0 - P.nst;
    return T;
}

// Issues the global loads of a tile's first column pass into reg: thread
// (chunk, col) gets rows chunk*CM .. chunk*CM+CM-1 of LDS column col.
// Words outside the page get the value that the input transform of
// take_loads turns into all ones.
__device__ __forceinline__ void issue_loads(const RectPage &P, const Tile &T, uint64_t (&reg)[CM])
{
    const int tid = threadIdx.x;
    const int chunk = tid / T.TW, col = tid - (tid / T.TW) * T.TW;
    const int chunks = (T.NR + CM - 1) / CM;
    const int a = chunk * CM;
    const int gj = T.gj0 + col;
    const bool colin = chunk < chunks && gj >= 0 && gj < P.nw;
    const uint64_t fill = P.in_c ? 0ull : kOnes;
    const uint64_t *p = T.src + (long long)(T.gy0 + a) * P.sstride + gj;
    const bool interior = T.gy0 >= 0 && T.gy0 + T.NR <= P.H;
    if (interior) {
#pragma unroll
        for (int i = 0; i < CM; i++) {
            reg[i] = (colin && a + i < T.NR) ? *p : fill;
            p += P.sstride;
        }
    } else {
#pragma unroll
        for (int i = 0; i < CM; i++) {
            const int gy = T.gy0 + a + i;
            reg[i] = (colin && a + i < T.NR && gy >= 0 && gy < P.H) ? *p : fill;
            p += P.sstride;
        }
    }
}

// Completes the loads: optional complement, pad bits of the last word set.
__device__ __forceinline__ void take_loads(const RectPage &P, const Tile &T, uint64_t (&reg)[CM])
{
    const int tid = threadIdx.x;
    const int col = tid - (tid / T.TW) * T.TW;
    const uint64_t inv = P.in_c ? kOnes : 0ull;
    const uint64_t pad = (T.gj0 + col == P.nw - 1) ? ~P.padmask : 0ull;
#pragma unroll
    for (int i = 0; i < CM; i++) reg[i] = (reg[i] ^ inv) | pad;
}


// Runs every stage of one tile.  reg holds the tile's first-stage loads
// (issued, not yet waited for).  Before the last row pass, which needs only
// LDS, the loads of the next tile are issued into reg, so they are in flight
// while this tile finishes.
template <int NST, int NT, class GetNext>
__device__ __forceinline__ bool process_tile(const RectPage &P, const Tile &T, uint64_t (&reg)[CM],
                                             uint64_t *lds, GetNext get_next)
{
    bool more = false;
    const int tid = threadIdx.x;
    constexpr int nst = NST;
    int NRs = T.NR;
    int gy0 = T.gy0;
    const int TWp = T.TWp;
#pragma unroll
    for (int s = 0; s < nst; s++) {
        const Stage S = (s == 0) ? P.st[0] : P.st[1];
        const bool last = s + 1 == nst;

        // ---- column pass (first: the order is free by separability)
        const int c_lo = s, ncols = T.TW - 2 * s;
        const int chunks = (NRs + CM - 1) / CM;
        const int rows = chunks * CM;
        const int chunk = tid / ncols;
        const int col = c_lo + (tid - chunk * ncols);
        const bool active = chunk < chunks;
        const int a = chunk * CM;
        if (s == 0) {
            take_loads(P, T, reg);
        } else {
            // inactive threads read the last row; their runs are never stored
            const int last = (rows - 1) * TWp + col;
            int idx = a * TWp + col;
#pragma unroll
            for (int i = 0; i < CM; i++) {
                reg[i] = lds[min(idx, last)];
                idx += TWp;
            }
        }
        const int h = S.h;
        int m = 1;
        if (h >= 2)  { col_step<1>(lds, reg, TWp, rows, col, a, active);  m = 2; }
        if (h >= 4)  { col_step<2>(lds, reg, TWp, rows, col, a, active);  m = 4; }
        if (h >= 8)  { col_step<4>(lds, reg, TWp, rows, col, a, active);  m = 8; }
        if (h >= 16) { col_step<8>(lds, reg, TWp, rows, col, a, active);  m = 16; }
        if (h >= 32) { col_step<16>(lds, reg, TWp, rows, col, a, active); m = 32; }
        while (2 * m <= h) {
            col_step_lds(lds, reg, TWp, rows, col, a, active, m);
            m *= 2;
        }
        if (h > m) col_step_lds(lds, reg, TWp, rows, col, a, active, h - m);
        const int NRo = NRs - (h - 1);  // rows of this stage's output
        const int gyo = gy0 + S.cy;     // page row of output row 0
        if (h > 1) lds_barrier();       // partners read: LDS free for the results
        if (active) {
#pragma unroll
            for (int i = 0; i < CM; i++) lds[(a + i) * TWp + col] = reg[i];
        }
        lds_barrier();

        // ---- row pass on rows [0, NRo): output columns [c_lo+1, TW-1-s)
        const int o_lo = c_lo + 1, o_hi = T.TW - 1 - s;
        const int G = (o_hi - o_lo + WPT - 1) / WPT;
        const int items = NRo * G;
        const int dr = NT / G, dg = NT - (NT / G) * G;
        if (last) {
            more = get_next(reg);           // issues the next tile's loads into reg
            const uint64_t inv = P.out_c ? kOnes : 0ull;
            int r = tid / G, g = tid - (tid / G) * G;
            for (int q = tid; q < items; q += NT) {
                const int c0 = o_lo + g * WPT;
                uint64_t X[WPT + 2];
                load_group(lds + r * TWp, c0, X);
                uint64_t o[WPT];
                if (S.w > 1) {
                    row_pass_group(X, S.w, S.cx, o);
                } else {
#pragma unroll
                    for (int i = 0; i < WPT; i++) o[i] = X[i + 1];
                }
                const int gj = T.gj0 + c0;
#pragma unroll
                for (int i = 0; i < WPT; i++) o[i] ^= inv;
                if (gj + WPT > P.nw - 1 && gj <= P.nw - 1) {
#pragma unroll
                    for (int i = 0; i < WPT; i++)
                        if (gj + i == P.nw - 1) o[i] &= P.padmask;
                }
                uint64_t *out = T.dst + (long long)(gyo + r) * P.dstride + gj;
                if (c0 + WPT <= o_hi && (((uintptr_t)out) & 15) == 0) {
                    ulonglong2 *o2 = reinterpret_cast<ulonglong2 *>(out);
#pragma unroll
                    for (int i = 0; i < WPT / 2; i++) o2[i] = make_ulonglong2(o[2 * i], o[2 * i + 1]);
                } else {
#pragma unroll
                    for (int i = 0; i < WPT; i++)
                        if (c0 + i < o_hi) out[i] = o[i];
                }
                r += dr;
                g += dg;
                if (g >= G) { g -= G; r++; }
            }
        } else {
            // intermediate: computed into registers, then written back in
            // place, (complemented,) clipped to the page with outside = 1
            // items here are taken rows fastest (every lane's results stay in
            // LDS): the 4-word groups of neighbouring lanes then start a row
            // pitch apart instead of 32 bytes, which spreads the row pass's
            // reads and the write-back over the banks
            uint64_t res[kItemsMax][WPT];
            const int dr2 = NT % NRo, dg2 = NT / NRo;
            int r = tid % NRo, g = tid / NRo;
#pragma unroll
            for (int k = 0; k < kItemsMax; k++) {
                if (tid + k * NT < items) {
                    const int c0 = o_lo + g * WPT;
                    uint64_t X[WPT + 2];
                    load_group(lds + r * TWp, c0, X);
                    if (S.w > 1) {
                        row_pass_group(X, S.w, S.cx, res[k]);
                    } else {
#pragma unroll
                        for (int i = 0; i < WPT; i++) res[k][i] = X[i + 1];
                    }
                }
                r += dr2;
                g += dg2;
                if (r >= NRo) { r -= NRo; g++; }
            }
            lds_barrier();
            r = tid % NRo;
            g = tid / NRo;
            const uint64_t minv = P.mid_c ? kOnes : 0ull;
#pragma unroll
            for (int k = 0; k < kItemsMax; k++) {
                if (tid + k * NT < items) {
                    const int c0 = o_lo + g * WPT;
                    const int gy = gyo + r;
                    const bool rowin = gy >= 0 && gy < P.H;
#pragma unroll
                    for (int i = 0; i < WPT; i++) {
                        const int c = c0 + i, gj = T.gj0 + c;
                        if (c < o_hi) {
                            uint64_t v = res[k][i] ^ minv;
                            if (!rowin || gj < 0 || gj >= P.nw) v = kOnes;
                            else if (gj == P.nw - 1) v |= ~P.padmask;
                            lds[r * TWp + c] = v;
                        }
                    }
                }
                r += dr2;
                g += dg2;
                if (r >= NRo) { r -= NRo; g++; }
            }
            lds_barrier();
            NRs = NRo;
            gy0 = gyo;
        }
    }
    return more;
}

// Tiles of a launch are numbered page-major, then band, then strip.  Each XCD
// (workgroups are dealt round-robin over the 8 XCDs) takes a contiguous range
// of tiles, so neighbouring tiles share halo rows in one L2.
__device__ __forceinline__ void tile_coords(const RectPage &P, int t, int &page, int &band, int &strip)
{
    const int per_page = P.nbands * P.nstrips;
    page = t / per_page;
    const int u = t - page * per_page;
    band = u / P.nstrips;
    strip = u - band * P.nstrips;
}

// One operation over all tiles of npages pages: a persistent grid, each
// workgroup taking every nx-th tile of its XCD's range.  Tile coordinates
// advance by carries, without divisions in the loop.
template <int NST, int NT>
__device__ __forceinline__ void rect_loop(const RectPage &P, uint64_t *lds, int ntiles)
{
    const int G = (int)gridDim.x, b = (int)blockIdx.x;
    const int x = b & 7, nx = (G - x + 7) >> 3;
    const int q = ntiles >> 3, rem = ntiles & 7;
    const int start = x * q + min(x, rem), count = q + (x < rem ? 1 : 0);
    int k = b >> 3;
    if (k >= count) return;
    const int nb = P.nbands, ns = P.nstrips;
    // step nx tiles = dp pages, db bands, ds strips (with carries)
    const int per_page = nb * ns;
    const int dp = nx / per_page, du = nx - dp * per_page;
    const int db = du / ns, ds = du - db * ns;
    int page, band, strip;
    tile_coords(P, start + k, page, band, strip);
    uint64_t reg[CM];
    issue_loads(P, make_tile(P, page, band, strip), reg);
    for (;;) {
        int np = page + dp, nbd = band + db, nst = strip + ds;
        if (nst >= ns) { nst -= ns; nbd++; }
        if (nbd >= nb) { nbd -= nb; np++; }
        const bool has = k + nx < count;
        auto get_next = [&](uint64_t (&r)[CM]) {
            if (!has) return false;
            issue_loads(P, make_tile(P, np, nbd, nst), r);
            return true;
        };
        if (!process_tile<NST, NT>(P, make_tile(P, page, band, strip), reg, lds, get_next)) break;
        k += nx;
        page = np;
        band = nbd;
        strip = nst;
        lds_barrier();
    }
}

template <int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) void rect_kernel(RectPage Parg, int ntiles)
{
    __shared__ __align__(16) uint64_t lds[lds_words_for(NT)];
    // the page parameters are read from the argument segment where they are
    // used, rather than all held in scalar registers for the whole kernel
    (void)Parg;
    const RectPage &P = *(const RectPage *)__builtin_amdgcn_kernarg_segment_ptr();
    if (P.nst == 1)
        rect_loop<1, NT>(P, lds, ntiles);
    else
        rect_loop<2, NT>(P, lds, ntiles);
}

// A batch of pages with their own operations: workgroups take tiles from a
// shared queue (largest pages first), claiming the next tile early so its
// loads can be issued before the current tile ends.
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4))) void rect_batch_kernel(
    const RectPage *__restrict__ pages, const TileRef *__restrict__ tiles, int ntiles, int *queue)
{
    __shared__ __align__(16) uint64_t lds[kLdsWords];
    __shared__ int slot[2];
    if (threadIdx.x == 0) slot[0] = atomicAdd(queue, 1);
    __syncthreads();
    int t = __builtin_amdgcn_readfirstlane(slot[0]);
    if (t >= ntiles) return;                       // every wave sees the same t
    uint64_t reg[CM];
    {
        const TileRef tr = tiles[t];
        const RectPage &P = pages[__builtin_amdgcn_readfirstlane(tr.page)];
        issue_loads(P, make_tile(P, 0, __builtin_amdgcn_readfirstlane(tr.band),
                                 __builtin_amdgcn_readfirstlane(tr.strip)), reg);
    }
    int parity = 1;
    for (;;) {
        // claim the next tile now; it is read after this tile's first barrier
        if (threadIdx.x == 0) slot[parity] = atomicAdd(queue, 1);
        const int par = parity;
        int tn = ntiles;
        auto get_next = [&](uint64_t (&r)[CM]) {
            tn = __builtin_amdgcn_readfirstlane(slot[par]);
            if (tn >= ntiles) return false;
            const TileRef r2 = tiles[tn];
            const RectPage &Pn = pages[__builtin_amdgcn_readfirstlane(r2.page)];
            issue_loads(Pn, make_tile(Pn, 0, __builtin_amdgcn_readfirstlane(r2.band),
                                      __builtin_amdgcn_readfirstlane(r2.strip)), r);
            return true;
        };
        const TileRef tr = tiles[t];
        const RectPage &P = pages[__builtin_amdgcn_readfirstlane(tr.page)];
        const Tile T = make_tile(P, 0, __builtin_amdgcn_readfirstlane(tr.band),
                                 __builtin_amdgcn_readfirstlane(tr.strip));
        const bool more = P.nst == 1 ? process_tile<1, kThreads>(P, T, reg, lds, get_next)
                                     : process_tile<2, kThreads>(P, T, reg, lds, get_next);
        if (!more) break;
        t = tn;
        parity ^= 1;
        lds_barrier();
    }
}

__global__ void reset_counter_kernel(int *q)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *q = 0;
}

int cached_cu_count = 0;


// ------------------------------------------------------------- transpose
// One workgroup of 256 threads per tile of kTrRows rows x kTrWords words of
// a page (blocks of 64 x 64 pixels).  Each thread loads whole tile rows,
// kTrWords contiguous words each, into LDS; then each wave turns the
// blocks of kTrWords / 4 word columns: for each it runs the butterfly on
// the kTrRows / 64 blocks below each other, after which lane i holds that
// many consecutive words of transposed row 64j + i and stores them
// contiguously.  Rows are padded by one word in LDS so that the column
// reads of the butterfly input spread over the banks.  (A persistent grid
// walking tile ranges, with the next tile's loads in flight during the
// butterflies, measured 1.4x slower on the letter batch.)
//
// With counts, each lane also counts the runs that start in its words of
// the transposed row (the pixel before them is bit i of the source row above
// the tile) and writes the count of its piece of the row to
// counts[tile row * rows + row] (a wave's 64 counts contiguous): the run
// counts of the transpose come with the transpose itself.
constexpr int kTrRows = 512, kTrWords = 8, kTrPad = kTrWords + 1;
constexpr int kTrRowsPerThread = kTrRows / 256, kTrColsPerWave = kTrWords / 4, kTrBlocks = kTrRows / 64;

struct TrTile {
    int page, tx, ty, y0, j0, nj;
};

__device__ __forceinline__ TrTile tr_tile(long long t, int tiles_y, int tiles_x, int nw)
{
    TrTile T;
    const long long per_page = (long long)tiles_y * tiles_x;
    T.page = (int)(t / per_page);
    const int u = (int)(t - (long long)T.page * per_page);
    T.tx = u / tiles_y;                 // row tiles fastest
    T.ty = u - T.tx * tiles_y;
    T.y0 = T.ty * kTrRows;
    T.j0 = T.tx * kTrWords;
    T.nj = min(kTrWords, nw - T.j0);
    return T;
}

// This thread's rows of a tile (words past the row or the page are 0, the
// row's pad bits cleared), and with `above` the word of the row above the
// tile for threads below kTrWords.
__device__ __forceinline__ void tr_load(const uint64_t *src, const TrTile &T, int H, int sstride, long long spw,
                                        uint64_t padmask, int nw, uint64_t (&v)[kTrRowsPerThread][kTrWords],
                                        uint64_t &ab, bool want_above)
{
    const uint64_t *sp = src + (long long)T.page * spw;
#pragma unroll
    for (int h = 0; h < kTrRowsPerThread; h++) {
        const int y = T.y0 + (int)threadIdx.x + 256 * h;
        const uint64_t *q = sp + (long long)y * sstride + T.j0;
        if (y < H && T.nj == kTrWords && (((uintptr_t)q) & 15) == 0) {
            const ulonglong2 *q2 = reinterpret_cast<const ulonglong2 *>(q);
#pragma unroll
            for (int c = 0; c < kTrWords / 2; c++) {
                const ulonglong2 w2 = q2[c];
                v[h][2 * c] = w2.x;
                v[h][2 * c + 1] = w2.y;
            }
        } else {
#pragma unroll
            for (int c = 0; c < kTrWords; c++) v[h][c] = (y < H && c < T.nj) ? q[c] : 0ull;
        }
        // the last word of the row: pad bits are 0 (a select per word: an
        // index computed at run time would put v in scratch memory)
#pragma unroll
        for (int c = 0; c < kTrWords; c++) v[h][c] &= (T.j0 + c == nw - 1) ? padmask : ~0ull;
    }
    ab = 0;
    if (want_above && threadIdx.x < kTrWords) {
        const int c = (int)threadIdx.x, y = T.y0 - 1;
        if (y >= 0 && c < T.nj) {
            ab = sp[(long long)y * sstride + T.j0 + c];
            if (T.j0 + c == nw - 1) ab &= padmask;
        }
    }
}

__global__ __launch_bounds__(256) void transpose_kernel(
    const uint64_t *__restrict__ src, int W, int H, int sstride, long long spw, uint64_t padmask,
    uint64_t *__restrict__ dst, int dstride, long long dpw, int nw, int nk, int tiles_y, int tiles_x,
    long long ntiles, int *__restrict__ counts)
{
    __shared__ uint64_t tile[kTrRows * kTrPad];
    __shared__ uint64_t above[kTrWords];
    const long long t = xcd_block();
    if (t >= ntiles) return;                // whole workgroup
    const bool cnt_on = counts != nullptr;
    const long long R = (long long)(ntiles / ((long long)tiles_y * tiles_x)) * W;   // transposed rows
    const int lane = (int)(threadIdx.x & 63), wv = (int)(threadIdx.x >> 6);
    const TrTile C = tr_tile(t, tiles_y, tiles_x, nw);
    uint64_t v[kTrRowsPerThread][kTrWords];
    uint64_t ab;
    tr_load(src, C, H, sstride, spw, padmask, nw, v, ab, cnt_on);
#pragma unroll
    for (int h = 0; h < kTrRowsPerThread; h++)
#pragma unroll
        for (int c = 0; c < kTrWords; c++) tile[((int)threadIdx.x + 256 * h) * kTrPad + c] = v[h][c];
    if (cnt_on && threadIdx.x < kTrWords) above[threadIdx.x] = ab;
    __syncthreads();
    const int nkk = min(kTrBlocks, nk - C.y0 / 64);        // row blocks of this tile
#pragma unroll
    for (int hc = 0; hc < kTrColsPerWave; hc++) {
        const int jj = kTrColsPerWave * wv + hc;         // word column of the tile
        uint64_t o[kTrBlocks];
#pragma unroll
        for (int kk = 0; kk < kTrBlocks; kk++) o[kk] = wave_transpose64(tile[(64 * kk + lane) * kTrPad + jj]);
        const int x = 64 * (C.j0 + jj) + lane;
        if (cnt_on) {                       // rows past the page bottom are 0
            uint64_t prev = (above[jj] >> lane) & 1ull;
            int cnt = 0;
#pragma unroll
            for (int kk = 0; kk < kTrBlocks; kk++) {
                cnt += __popcll(o[kk] & ~((o[kk] << 1) | prev));
                prev = o[kk] >> 63;
            }
            if (jj < C.nj && x < W) counts[(long long)C.ty * R + (long long)C.page * W + x] = cnt;
        }
        if (jj < C.nj && x < W) {
            uint64_t *dp = dst + (long long)C.page * dpw + (long long)x * dstride + C.y0 / 64;
            if (nkk == kTrBlocks && (((uintptr_t)dp) & 15) == 0) {
                ulonglong2 *q = reinterpret_cast<ulonglong2 *>(dp);
#pragma unroll
                for (int c = 0; c < kTrBlocks / 2; c++) q[c] = make_ulonglong2(o[2 * c], o[2 * c + 1]);
            } else {
#pragma unroll
                for (int kk = 0; kk < kTrBlocks; kk++)
                    if (kk < nkk) dp[kk] = o[kk];
            }
        }
    }
}


// ----------------------------------------------------------- arbitrary masks
// Erosion by an arbitrary mask, one workgroup per tile of TR rows x SW
// words (section "Morphology with Arbitrary Masks", the doubling
// accumulation): the tile's input rows with their halo are loaded into LDS
// (outside pixels 1), the horizontal erosions by 1, 2, 4, ... pixels are
// built in LDS level by level, and every output word is the AND over the
// mask's runs of the erosion by the run's length, taken from the largest
// level not longer than the run at the run's two ends, shifted by the run's
// offsets.
constexpr int kMaskLdsWords = 4096;     // 32 KiB of levels per workgroup (4 per CU)

// The 64 bits from bit position p of an LDS row of nwords words (1s past it).
__device__ __forceinline__ uint64_t lds_bits(const uint64_t *row, int nwords, int p)
{
    const int w = p >> 6, s = p & 63;
    if (w >= nwords) return kOnes;
    const uint64_t lo = row[w];
    if (s == 0) return lo;
    const uint64_t hi = (w + 1 < nwords) ? row[w + 1] : kOnes;
    return funnel_r(hi, lo, s);
}

__global__ __launch_bounds__(256) void mask_kernel(MaskPage P, MaskRunsArg M, long long ntiles)
{
    extern __shared__ uint64_t lv[];        // levels x NR x NW
    const long long t = xcd_block();
    if (t >= ntiles) return;                // whole workgroup
    const long long per_page = (long long)P.nbands * P.nstrips;
    const int page = (int)(t / per_page);
    const int u = (int)(t - (long long)page * per_page);
    const int band = u / P.nstrips, strip = u - band * P.nstrips;
    const int y0 = band * P.TR, j0 = strip * P.SW;
    const int TRv = min(P.TR, P.H - y0), SWv = min(P.SW, P.nw - j0);
    const int NR = P.NR, NW = P.NW, plane = NR * NW;
    const uint64_t inv = P.in_c ? kOnes : 0ull;
    const uint64_t *sp = P.src + (long long)page * P.spw;
    for (int i = threadIdx.x; i < plane; i += 256) {
        const int r = i / NW, w = i - r * NW;
        const int y = y0 + P.dy0 + r, j = j0 - P.HL + w;
        uint64_t v = kOnes;
        if (y >= 0 && y < P.H && j >= 0 && j < P.nw) {
            v = sp[(long long)y * P.sstride + j] ^ inv;
            if (j == P.nw - 1) v |= ~P.padmask;
        }
        lv[i] = v;
    }
    __syncthreads();
    for (int l = 1; l < P.levels; l++) {    // E_{2^l}(x) = E_{2^(l-1)}(x) & E_{2^(l-1)}(x + 2^(l-1))
        const uint64_t *prev = lv + (long long)(l - 1) * plane;
        uint64_t *cur = lv + (long long)l * plane;
        const int k = 1 << (l - 1);
        for (int i = threadIdx.x; i < plane; i += 256) {
            const int r = i / NW, w = i - r * NW;
            cur[i] = prev[i] & lds_bits(prev + r * NW, NW, 64 * w + k);
        }
        __syncthreads();
    }
    const uint64_t outv = P.out_c ? kOnes : 0ull;
    uint64_t *dp = P.dst + (long long)page * P.dpw;
    for (int i = threadIdx.x; i < TRv * SWv; i += 256) {
        const int r = i / SWv, c = i - r * SWv;
        const int pbase = 64 * (c + P.HL);
        uint64_t acc = kOnes;
        for (int q = 0; q < M.n; q++) {
            const int len = M.len[q];
            const int l = 31 - __clz(len), m = 1 << l;
            const uint64_t *row = lv + (long long)l * plane + (r + M.dy[q] - P.dy0) * NW;
            const int p = pbase + M.dx[q];
            acc &= lds_bits(row, NW, p) & lds_bits(row, NW, p + len - m);
        }
        const int j = j0 + c;
        uint64_t o = acc ^ outv;
        if (j == P.nw - 1) o &= P.padmask;
        dp[(long long)(y0 + r) * P.dstride + j] = o;
    }
}


// ---------------------------------------------------------------- line shifts
// Every line moves right by its own shift (section "Scaling, Skewing, and
// Rotation": skews are shifts within lines): dst(x, y) = src(x - shift[y], y)
// inside the source, fill elsewhere.  One thread per output word: the two
// source words under it, a funnel shift, then the fill outside the source
// and 0 in the destination's pad bits.
__global__ __launch_bounds__(256) void shift_rows_kernel(const uint64_t *__restrict__ src, int Ws, int nws, int sstride,
                                                         uint64_t *__restrict__ dst, int Wd, int nwd, int dstride,
                                                         const int *__restrict__ shifts, int fill, long long total)
{
    const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
    if (t >= total) return;
    const long long r = t / nwd;
    const int j = (int)(t - r * nwd);
    const long long sh = min(max((long long)shifts[r], -(1LL << 30)), 1LL << 30);
    const uint64_t fw = fill ? kOnes : 0ull;
    const uint64_t *row = src + r * sstride;
    const long long p = 64LL * j - sh;      // source bit under the word's bit 0
    const long long q = p >> 6;             // floor
    const int b = (int)(p & 63);
    auto word = [&](long long k) { return (k >= 0 && k < nws) ? row[k] : fw; };
    const uint64_t lo = word(q);
    const uint64_t v = b == 0 ? lo : funnel_r(word(q + 1), lo, b);
    // bits of the word whose source lies in [0, Ws)
    const long long x0 = 64LL * j;
    const long long a = max(sh, x0) - x0, e = min(sh + Ws, x0 + 64) - x0;
    uint64_t valid = 0;
    if (a < e) valid = (~0ull >> (64 - (e - a))) << a;
    uint64_t o = (v & valid) | (fw & ~valid);
    const int rem = Wd - 64 * j;            // pad bits of the destination
    if (rem < 64) o &= (1ull << rem) - 1;
    dst[r * dstride + j] = o;
}


// ------------------------------------------------------------ pixel counts
// Black pixels per page, the input of the choice between the packed and the
// run-length path: counts[page] is cleared by block 0 of the first launch,
// then every workgroup adds the popcount of a range of rows of one page
// (pad bits masked off) with one 64-bit atomic.
__global__ void clear_counts_kernel(unsigned long long *counts, int n)
{
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i < n) counts[i] = 0ull;
}

__global__ __launch_bounds__(256) void popcount_kernel(const uint64_t *__restrict__ src, int nw, int stride, int H,
                                                      long long page_words, uint64_t padmask, int rows_per_block,
                                                      int blocks_per_page, unsigned long long *counts)
{
    __shared__ unsigned long long part[4];
    const int page = (int)(blockIdx.x / (unsigned)blocks_per_page);
    const int blk = (int)(blockIdx.x - (unsigned)page * (unsigned)blocks_per_page);
    const int y0 = blk * rows_per_block, y1 = min(H, y0 + rows_per_block);
    const uint64_t *p = src + (long long)page * page_words;
    unsigned long long c = 0;
    const long long n = (long long)(y1 - y0) * nw;
    for (long long i = threadIdx.x; i < n; i += 256) {
        const int y = y0 + (int)(i / nw), j = (int)(i - (long long)(y - y0) * nw);
        uint64_t v = p[(long long)y * stride + j];
        if (j == nw - 1) v &= padmask;
        c += (unsigned long long)__popcll(v);
    }
    for (int o = 32; o > 0; o >>= 1) c += __shfl_down(c, o, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned long long t = part[0] + part[1] + part[2] + part[3];
        if (t) atomicAdd(counts + page, t);
    }
}

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

// Largest number of rows (input rows of the first stage) a tile of width TW
// can hold for page p, or 0 if none: the LDS array (rows are allocated in
// runs of kChunkMax at the pitch of tile_pitch, 8 words of slack), the
// column runs (one thread per run, so runs per column <= threads / columns),
// and the row-pass results a thread holds across a barrier in every stage
// but the last.
static int max_rows(const RectPage &p, int TW)
{
    const int TWp = tile_pitch(TW, p.nst);
    const int nthreads = p.nt;
    int nr = ((lds_words_for(p.nt) - 8) / TWp) / kChunkMax * kChunkMax;
    int drop = 0;                   // rows consumed before stage s
    for (int s = 0; s < p.nst; s++) {
        const int ncols = TW - 2 * s;
        if (ncols < 3) return 0;
        const int chunks = nthreads / ncols;
        if (chunks < 1) return 0;
        nr = std::min(nr, chunks * kChunkMax + drop);
        drop += p.st[s].h - 1;
        if (s + 1 < p.nst) {
            const int G = (ncols - 2 + WPT - 1) / WPT;
            nr = std::min(nr, (nthreads * kItemsMax) / G + drop);
        }
    }
    return nr;
}

bool plan_tiles(RectPage &p, int tile_rows, int strip_words, int npages, int nt)
{
    if (nt != kThreads && nt != kThreadsSmall) return false;
    p.nt = nt;
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
        const long long want = (long long)(2 * kThreads / nt) * device_cu_count();
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
    if (p.nt != kThreads && p.nt != kThreadsSmall) return false;
    const int nthreads = p.nt;
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
    const int TWp = tile_pitch(TW, p.nst);
    int NRs = p.TR + hsum;
    const int rows0 = (NRs + kChunkMax - 1) / kChunkMax * kChunkMax;
    if ((long long)rows0 * TWp + 8 > lds_words_for(p.nt)) return false;
    for (int s = 0; s < p.nst; s++) {
        const int ncols = TW - 2 * s;
        if (ncols < 3) return false;
        if ((NRs + kChunkMax - 1) / kChunkMax > nthreads / ncols) return false;
        NRs -= p.st[s].h - 1;
        if (NRs < 1) return false;
        if (s + 1 < p.nst &&
            (long long)NRs * ((ncols - 2 + WPT - 1) / WPT) > (long long)nthreads * kItemsMax)
            return false;
    }
    return true;
}

hipError_t launch_rect(const RectPage &p, int npages, hipStream_t stream)
{
    const long long T = (long long)p.nbands * p.nstrips * npages;
    if (T <= 0) return hipSuccess;
    if (!tile_fits(p) || T > 0x7fffffffLL) return hipErrorInvalidValue;
    const int grid = (int)std::min<long long>(T, (long long)(2 * kThreads / p.nt) * device_cu_count());
    trace_before(MORPH_K_RECT, stream);
    if (p.nt == kThreadsSmall)
        hipLaunchKernelGGL(rect_kernel<kThreadsSmall>, dim3(grid), dim3(kThreadsSmall), 0, stream, p, (int)T);
    else
        hipLaunchKernelGGL(rect_kernel<kThreads>, dim3(grid), dim3(kThreads), 0, stream, p, (int)T);
    trace_after(MORPH_K_RECT, stream, 16.0 * p.nw * (double)p.H * npages);
    return hipGetLastError();
}

hipError_t launch_rect_batch(const RectPage *pages_dev, const TileRef *tiles_dev, int ntiles,
                             int *queue_dev, int nblocks, hipStream_t stream, double alg_bytes)
{
    trace_before(MORPH_K_RECT_BATCH, stream);
    hipLaunchKernelGGL(rect_batch_kernel, dim3(nblocks), dim3(kThreads), 0, stream, pages_dev,
                       tiles_dev, ntiles, queue_dev);
    trace_after(MORPH_K_RECT_BATCH, stream, alg_bytes);
    return hipGetLastError();
}

static hipError_t launch_transpose(const morph_bitmap_t &dst, const morph_bitmap_t &src, int *counts,
                                   hipStream_t stream)
{
    const int W = src.width, H = src.height;
    const int nw = (W + 63) / 64, nk = (H + 63) / 64;
    const int tiles_y = (H + kTrRows - 1) / kTrRows, tiles_x = (nw + kTrWords - 1) / kTrWords;
    const long long ntiles = (long long)tiles_y * tiles_x * src.npages;
    if (ntiles <= 0) return hipSuccess;
    if (ntiles > 0x7fffffffLL) return hipErrorInvalidValue;
    const uint64_t pad = (W % 64) ? ((1ull << (W % 64)) - 1) : ~0ull;
    hipLaunchKernelGGL(transpose_kernel, dim3((unsigned)ntiles), dim3(256), 0, stream, src.words, W, H,
                       src.stride_words, (long long)src.stride_words * H, pad, dst.words, dst.stride_words,
                       (long long)dst.stride_words * W, nw, nk, tiles_y, tiles_x, ntiles, counts);
    return hipGetLastError();
}

hipError_t packed_transpose(const morph_bitmap_t &dst, const morph_bitmap_t &src, hipStream_t stream)
{
    const int nw = (src.width + 63) / 64, nk = (src.height + 63) / 64;
    trace_before(MORPH_K_TRANSPOSE, stream);
    const hipError_t e = launch_transpose(dst, src, nullptr, stream);
    trace_after(MORPH_K_TRANSPOSE, stream, 8.0 * src.npages * ((double)nw * src.height + (double)nk * src.width));
    return e;
}

int transpose_pieces(int height) { return (height + kTrRows - 1) / kTrRows; }

hipError_t packed_transpose_counted(const morph_bitmap_t &dst, const morph_bitmap_t &src, int *counts,
                                    hipStream_t stream)
{
    return launch_transpose(dst, src, counts, stream);
}

bool plan_mask(MaskPage &p, const MaskRunsArg &m)
{
    int dxmin = 0, reach = 0, dymin = 0, dymax = 0, maxlen = 1;
    for (int q = 0; q < m.n; q++) {
        if (m.len[q] < 1) return false;
        dxmin = std::min(dxmin, (int)m.dx[q]);
        reach = std::max(reach, m.dx[q] + m.len[q] - 1);
        dymin = std::min(dymin, (int)m.dy[q]);
        dymax = std::max(dymax, (int)m.dy[q]);
        maxlen = std::max(maxlen, (int)m.len[q]);
    }
    int levels = 1;
    while ((2 << (levels - 1)) <= maxlen) levels++;
    p.HL = (-dxmin + 63) / 64;
    p.HR = (reach + 63) / 64;
    p.dy0 = dymin;
    p.levels = levels;
    int SW = std::min(p.nw, 8), TR = 64;
    for (;;) {
        p.NR = TR + dymax - dymin;
        p.NW = SW + p.HL + p.HR;
        if ((long long)levels * p.NR * p.NW <= kMaskLdsWords) break;
        if (TR > 8) TR /= 2;
        else if (SW > 1) SW /= 2;
        else if (TR > 1) TR /= 2;
        else return false;
    }
    p.TR = TR;
    p.SW = SW;
    p.nbands = (p.H + TR - 1) / TR;
    p.nstrips = (p.nw + SW - 1) / SW;
    return true;
}

hipError_t launch_mask(const MaskPage &p, const MaskRunsArg &m, int npages, hipStream_t stream)
{
    const long long ntiles = (long long)p.nbands * p.nstrips * npages;
    if (ntiles <= 0) return hipSuccess;
    if (ntiles > 0x7fffffffLL) return hipErrorInvalidValue;
    const size_t lds = (size_t)p.levels * p.NR * p.NW * sizeof(uint64_t);
    trace_before(MORPH_K_MASK, stream);
    hipLaunchKernelGGL(mask_kernel, dim3((unsigned)ntiles), dim3(256), lds, stream, p, m, ntiles);
    trace_after(MORPH_K_MASK, stream, 16.0 * p.nw * (double)p.H * npages);
    return hipGetLastError();
}

hipError_t shift_rows_packed(const morph_bitmap_t &dst, const morph_bitmap_t &src, const int *shifts, int fill,
                             hipStream_t stream)
{
    const long long R = (long long)src.height * src.npages;
    const int nws = (src.width + 63) / 64, nwd = (dst.width + 63) / 64;
    const long long total = R * nwd;
    if (total <= 0) return hipSuccess;
    if ((total + 255) / 256 > 0x7fffffffLL) return hipErrorInvalidValue;
    trace_before(MORPH_K_SHIFT, stream);
    hipLaunchKernelGGL(shift_rows_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, stream, src.words,
                       src.width, nws, src.stride_words, dst.words, dst.width, nwd, dst.stride_words, shifts, fill,
                       total);
    trace_after(MORPH_K_SHIFT, stream, 8.0 * R * ((double)nws + nwd) + 4.0 * R);
    return hipGetLastError();
}

hipError_t popcount_pages(const morph_bitmap_t &src, unsigned long long *counts, hipStream_t stream)
{
    const int P = src.npages, H = src.height, nw = (src.width + 63) / 64;
    const uint64_t pad = (src.width % 64) ? ((1ull << (src.width % 64)) - 1) : ~0ull;
    hipLaunchKernelGGL(clear_counts_kernel, dim3((P + 255) / 256), dim3(256), 0, stream, counts, P);
    // about 1024 workgroups over the stack, at least 8 rows each
    const int per_page = std::max(1, std::min((H + 7) / 8, (1024 + P - 1) / P));
    const int rows = (H + per_page - 1) / per_page;
    const int bpp = (H + rows - 1) / rows;
    const long long blocks = (long long)bpp * P;
    if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
    hipLaunchKernelGGL(popcount_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, src.words, nw,
                       src.stride_words, H, (long long)src.stride_words * H, pad, rows, bpp, counts);
    return hipGetLastError();
}

hipError_t launch_reset_counter(int *queue_dev, hipStream_t stream)
{
    hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(64), 0, stream, queue_dev);
    return hipGetLastError();
}

}  // namespace morph
