// Binning and sorting (TC-GS paper, Sec. 3.1 "Sorting"): per-tile splat
// lists ordered by depth, then Gaussian id.
//
// Instead of one radix sort of N 64-bit (tile | depth) keys, the stage
//   1. sorts the P Gaussians by depth (stable LSD radix, 4 x 8-bit passes on
//      an order-preserving image of the float bits; ties keep id order; the
//      first pass drops the Gaussians without splats),
//   2. scans the per-Gaussian tile counts in that order and expands the
//      splats (tile, id) in depth order, load-balanced over fixed windows of
//      output slots,
//   3. sorts the N splats by tile only (stable LSD radix over
//      ceil(log2 ntiles) bits in passes of near-equal width), which keeps
//      depth order within a tile, and
//   4. finds each tile's [start, end).
// Every splat moves 2 x (4 + 4) bytes per tile pass instead of 6 passes of
// 24 bytes.  A Gaussian covers the tiles of its 3-sigma pixel rectangle, or,
// with the precise rule (gs_bin_sort_precise), only those of them where its
// raw opacity can reach the culling threshold.  One call can serve several
// views of a scene (gs_bin_sort_multiview): every stage then runs over all
// (Gaussian, view) pairs, and the two sorts over per-view segments.
#include "common.h"

#include <mutex>

namespace {

constexpr int SORT_THREADS = 256;
// the counts and scan kernels: blocks of SORT_TILE counts, COUNT_THREADS
// threads of SORT_ITEMS each
constexpr int COUNT_THREADS = 512;
constexpr int SORT_ITEMS = 8;
constexpr int SORT_TILE = COUNT_THREADS * SORT_ITEMS;
constexpr int RADIX_BITS = 8;
constexpr int RADIX = 1 << RADIX_BITS;
constexpr int WAVES = SORT_THREADS / 64;
// keys per thread of a radix pass: the P Gaussians' depth sort runs twice as
// many (smaller) workgroups as the N splats' tile sort
constexpr int DEPTH_ITEMS = 8;
constexpr int TILE_ITEMS = 16;
// a one-view call with room for this many splats sorts them by tile in
// blocks of twice as many keys (longer runs of equal digits per block to
// write; below it, more and shorter blocks measure faster)
constexpr int TILE_ITEMS_BIG = 32;
constexpr uint32_t BIG_SORT_CAP = 24u << 20;
// 3-sigma expansion: windows of EMIT_TILE output slots, 512 threads of 4
// slots each (the window's staged Gaussians fill 33 KB of LDS, so wider
// workgroups are what keeps more waves per CU in flight)
constexpr int EMIT_THREADS = 512;
constexpr int EMIT_ITEMS = 4;
constexpr int EMIT_TILE = EMIT_THREADS * EMIT_ITEMS;
// precise rule: windows of 512 threads x 2 slots, with a table of up to
// RCAP (Gaussian, tile row) runs per window
constexpr int EMIT_THREADS_P = 512;
constexpr int EMIT_ITEMS_P = 2;
constexpr int EMIT_TILE_P = EMIT_THREADS_P * EMIT_ITEMS_P;
constexpr int RCAP = 1280;

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// ---------------------------------------------------------------------------
// Block-level scans
// ---------------------------------------------------------------------------
template <typename T> __device__ __forceinline__ T wave_incl_scan(T v) {
    int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        T o = __shfl_up(v, d, 64);
        if (lane >= d) v += o;
    }
    return v;
}

// Block-wide exclusive scan of one value per thread; returns the block total.
// `lds` needs blockDim.x / 64 entries.
template <typename T> __device__ __forceinline__ T block_excl_scan(T v, T &excl, T *lds) {
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    T inc = wave_incl_scan(v);
    if (lane == 63) lds[w] = inc;
    __syncthreads();
    T off = 0, tot = 0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) {
        T s = lds[i];
        if (i < w) off += s;
        tot += s;
    }
    excl = off + inc - v;
    __syncthreads();
    return tot;
}

// ---------------------------------------------------------------------------
// Device-wide exclusive scan of the per-Gaussian splat counts (u64 running
// totals so that an overflowing count is detected instead of wrapping): the
// counts kernel leaves one partial sum per block of SORT_TILE counts; each
// down-sweep block adds up the partials before it and the grand total N
// itself (block 0 publishes N), scans its counts, and records, for every
// window of `win` output slots, the Gaussian that owns the window's first
// slot.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(COUNT_THREADS) void k_scan_down(const uint32_t *__restrict__ cnt,
                                                            uint32_t *__restrict__ offs, uint32_t n,
                                                            const uint64_t *__restrict__ part,
                                                            uint32_t nparts,
                                                            uint32_t *__restrict__ win_start,
                                                            uint32_t nwin, int wshift,
                                                            uint32_t *__restrict__ d_total,
                                                            uint32_t *__restrict__ seg_bounds,
                                                            int nv, uint32_t Pv) {
    const uint64_t win = 1ull << wshift;  // window size (a power of two)
    __shared__ uint64_t lds[COUNT_THREADS / 64];
    // the block partials before this block, and all of them
    uint64_t before = 0, all = 0;
    for (uint32_t i0 = threadIdx.x; i0 < nparts; i0 += 4 * COUNT_THREADS) {
        uint64_t v[4];  // four loads in flight (index clamped; nparts >= 1 here)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const uint32_t i = i0 + r * COUNT_THREADS;
            v[r] = part[i < nparts ? i : nparts - 1];
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const uint32_t i = i0 + r * COUNT_THREADS;
            if (i < nparts) {
                all += v[r];
                before += i < blockIdx.x ? v[r] : 0ull;
            }
        }
    }
    uint64_t ex0;
    const uint64_t pre = block_excl_scan<uint64_t>(before, ex0, lds);
    const uint64_t N = block_excl_scan<uint64_t>(all, ex0, lds);
    const uint32_t Nsat = N > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)N;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        *d_total = Nsat;
        seg_bounds[nv] = Nsat;
    }
    size_t base = (size_t)blockIdx.x * SORT_TILE + (size_t)threadIdx.x * SORT_ITEMS;
    static_assert(SORT_ITEMS % 4 == 0, "16-byte loads");
    uint32_t v[SORT_ITEMS];
    uint64_t s = 0;
    if (base + SORT_ITEMS <= n) {  // (cnt is 256-byte aligned, base a multiple of SORT_ITEMS)
#pragma unroll
        for (int k = 0; k < SORT_ITEMS; k += 4) {
            const uint4 q = *(const uint4 *)(cnt + base + k);
            v[k] = q.x;
            v[k + 1] = q.y;
            v[k + 2] = q.z;
            v[k + 3] = q.w;
        }
    } else {
#pragma unroll
        for (int k = 0; k < SORT_ITEMS; ++k) v[k] = base + k < n ? cnt[base + k] : 0u;
    }
#pragma unroll
    for (int k = 0; k < SORT_ITEMS; ++k) s += v[k];
    uint64_t ex;
    block_excl_scan<uint64_t>(s, ex, lds);
    uint64_t run = pre + ex;
    // the thread's offsets: four 16-byte stores when all its items exist
    const bool full = base + SORT_ITEMS <= n;
    if (full) {
        uint32_t o[SORT_ITEMS];
        uint64_t r = run;
#pragma unroll
        for (int k = 0; k < SORT_ITEMS; ++k) {
            o[k] = (uint32_t)r;
            r += v[k];
        }
#pragma unroll
        for (int k = 0; k < SORT_ITEMS; k += 4)
            *(uint4 *)(offs + base + k) = make_uint4(o[k], o[k + 1], o[k + 2], o[k + 3]);
    }
    // view v's splats start at the offset of its first instance, v * Pv
    uint32_t vnext = (uint32_t)((base + Pv - 1) / Pv);
#pragma unroll
    for (int k = 0; k < SORT_ITEMS; ++k) {
        if (base + k < n) {
            if (!full) offs[base + k] = (uint32_t)run;
            if ((int)vnext < nv && base + k == (size_t)vnext * Pv) {
                seg_bounds[vnext] = run > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)run;
                ++vnext;
            }
            // windows whose first slot falls inside [run, run + v)
            if (v[k] > 0) {
                uint64_t w0 = (run + win - 1) >> wshift;
                uint64_t w1 = (run + v[k] - 1) >> wshift;
                for (uint64_t w = w0; w <= w1 && w < nwin; ++w) win_start[w] = (uint32_t)(base + k);
                // the owner of the last slot closes the last window
                uint64_t wl = (N + win - 1) >> wshift;
                if (run + v[k] == N && wl < nwin) win_start[wl] = (uint32_t)(base + k);
            }
        }
        run += v[k];
    }
}

// ---------------------------------------------------------------------------
// Stable LSD radix sort pass (BITS-bit digit, BITS <= 8) of u32 keys with u32
// values over independent segments of the arrays (the views of a multi-view
// frame; one segment for a single image): per-block digit histograms ->
// per-(segment, digit) scan over the segment's blocks -> scatter.  Each
// segment is split into blocks of TILE keys (the kernels' NT threads times
// ITEMS keys each); workgroup b of a launch takes block b of the
// concatenation of the segments' blocks (idle past the last one), so one
// launch serves every segment.
// ---------------------------------------------------------------------------
// With DROP, keys equal to DROP_KEY are left out (counted nowhere, written
// nowhere): the pass also compacts.
constexpr uint32_t DROP_KEY = 0xFFFFFFFFu;
constexpr int MAX_SEGS = GS_MAX_BIN_VIEWS;

// Segment s holds keys [base_s, base_s + n_s) of the arrays: base_s = s *
// stride and n_s = n_dev[s] (or n_static), or base_s = bounds[s] and n_s =
// bounds[s + 1] - bounds[s].  With `total`, every segment is empty when
// *total > cap (an overflowing frame).  The digit of a key in segment s is
// taken from key - kv[s].tbase (key itself without kv).
struct ViewDims {
    int W, H;
    uint32_t gx, tbase;
};

struct SegTable {
    int nseg;
    uint32_t stride, n_static;
    const uint32_t *n_dev;
    const uint32_t *bounds;
    const uint32_t *total;
    uint32_t cap;
    const ViewDims *kv;
    __device__ __forceinline__ uint32_t key_base(int sg) const { return kv ? kv[sg].tbase : 0u; }
    __device__ __forceinline__ void get(int sg, uint32_t &base, uint32_t &n) const {
        // independent loads (the pointers are uniform), then the selection
        uint32_t b0 = 0u, b1 = 0u, nd = n_static, tot = 0u;
        if (bounds) {
            b0 = bounds[sg];
            b1 = bounds[sg + 1];
        }
        if (n_dev) nd = n_dev[sg];
        if (total) tot = *total;
        base = bounds ? b0 : (uint32_t)sg * stride;
        n = bounds ? b1 - b0 : nd;
        if (total && tot > cap) {
            base = 0u;
            n = 0u;
        }
    }
};

// Segment, block within it, and the segment's range for workgroup b; false
// past the last block.  col0 = the segment's first workgroup.
template <int TILE>
__device__ __forceinline__ bool seg_block(const SegTable &st, uint32_t b, int &sg, uint32_t &lb,
                                          uint32_t &base, uint32_t &n, uint32_t &col0) {
    uint32_t acc = 0;
    for (int q = 0; q < st.nseg; ++q) {
        st.get(q, base, n);
        const uint32_t nb = (n + TILE - 1) / TILE;
        if (b < acc + nb) {
            sg = q;
            lb = b - acc;
            col0 = acc;
            return true;
        }
        acc += nb;
    }
    return false;
}

// Logical block of workgroup b of a radix launch: the launch's active blocks
// (the concatenated segments') are cut into 8 contiguous runs, run x served
// by XCD x (workgroups reach the 8 XCDs round-robin), so blocks whose
// output ranges neighbour each other (a digit's keys of block k are written
// just before those of block k + 1) share an L2 and their partial cache
// lines merge there.  False for padding workgroups.
template <int TILE>
__device__ __forceinline__ bool xcd_block(const SegTable &st, uint32_t b, uint32_t &lb) {
    uint32_t total = 0;
    for (int q = 0; q < st.nseg; ++q) {
        uint32_t base, n;
        st.get(q, base, n);
        total += (n + TILE - 1) / TILE;
    }
    const uint32_t per = (total + 7) / 8, j = b >> 3, x = b & 7;
    if (j >= per) return false;
    lb = x * per + j;
    return lb < total;
}

template <int ITEMS, int BITS, bool DROP, int NT, typename K = uint32_t>
__global__ __launch_bounds__(NT) void k_radix_hist(const K *__restrict__ keys,
                                                             SegTable st, int shift,
                                                             uint32_t *__restrict__ hist,
                                                             uint32_t ncols) {
    constexpr int NDIG = 1 << BITS;
    constexpr int TILE = NT * ITEMS;
    __shared__ uint32_t h[NDIG];
    int sg;
    uint32_t lb, base, n, col0, L;
    if (!xcd_block<TILE>(st, blockIdx.x, L)) return;  // idle: uniform exit
    if (!seg_block<TILE>(st, L, sg, lb, base, n, col0)) return;
    const uint32_t kb = st.key_base(sg);
    const size_t b0 = (size_t)lb * TILE;
    // every load issued before the first count (a block that is not idle has
    // n >= 1, so the index is clamped into the segment), then the counts
    uint32_t kv[ITEMS];
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
        const size_t i = b0 + (size_t)k * NT + threadIdx.x;
        kv[k] = keys[base + (i < n ? i : (size_t)n - 1)];
    }
    if (threadIdx.x < NDIG) h[threadIdx.x] = 0;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
        const size_t i = b0 + (size_t)k * NT + threadIdx.x;
        if (i < n && (!DROP || kv[k] != DROP_KEY))
            atomicAdd(&h[((kv[k] - kb) >> shift) & (NDIG - 1)], 1u);
    }
    __syncthreads();
    if (threadIdx.x < NDIG) hist[(size_t)threadIdx.x * ncols + L] = h[threadIdx.x];
}

// Exclusive scan over columns [0, nb) of get(i) into out[i], ROW_RPT
// consecutive columns per thread per round (a row of a few thousand blocks
// takes a few rounds, not one block scan per 256 columns); returns the
// total.  get(i) is called with i < nb only, and every column of a round
// is read before any is written, so out may be the row that get reads.
// All threads of the block call it.
constexpr int ROW_RPT = 8;
template <typename Get>
__device__ __forceinline__ uint32_t scan_columns(Get get, uint32_t *out, uint32_t nb,
                                                 uint32_t *lds) {
    uint32_t carry = 0;
    for (uint32_t c0 = 0; c0 < nb; c0 += SORT_THREADS * ROW_RPT) {
        const uint32_t i0 = c0 + threadIdx.x * ROW_RPT;
        uint32_t v[ROW_RPT], sum = 0;
#pragma unroll
        for (int r = 0; r < ROW_RPT; ++r) {
            const uint32_t i = i0 + r;
            const uint32_t x = get(i < nb ? i : nb - 1u);
            v[r] = i < nb ? x : 0u;
            sum += v[r];
        }
        uint32_t ex;
        const uint32_t tot = block_excl_scan<uint32_t>(sum, ex, lds);
        uint32_t run = carry + ex;
#pragma unroll
        for (int r = 0; r < ROW_RPT; ++r) {
            if (i0 + (uint32_t)r < nb) out[i0 + r] = run;
            run += v[r];
        }
        carry += tot;
    }
    return carry;
}

// Workgroup (d, s): exclusive scan of digit d's counts over the blocks of
// segment s, in place; the total goes to totals[s][d].  ncols = workgroups
// of the hist and scatter launches.
template <int TILE>
__global__ __launch_bounds__(SORT_THREADS) void k_hist_rows(uint32_t *__restrict__ hist,
                                                            SegTable st, uint32_t ncols,
                                                            uint32_t *__restrict__ totals) {
    __shared__ uint32_t lds[WAVES];
    const int sg = blockIdx.y;
    uint32_t col0 = 0, base, n;
    for (int q = 0; q < sg; ++q) {
        st.get(q, base, n);
        col0 += (n + TILE - 1) / TILE;
    }
    st.get(sg, base, n);
    const uint32_t nb = (n + TILE - 1) / TILE;
    uint32_t *row = hist + (size_t)blockIdx.x * ncols + col0;
    const uint32_t carry = scan_columns([&](uint32_t i) { return row[i]; }, row, nb, lds);
    if (threadIdx.x == 0) totals[sg * RADIX + blockIdx.x] = carry;
}

// With DROP, the first block of each segment also writes the number of keys
// the segment keeps to n_kept[s].  NT threads of ITEMS keys per block.
//
// With RANGES (the last pass of the tile sort, whose keys are the final
// tile order), the sorted keys are not written: the pass records where each
// tile starts, in ranges[2 t], instead.  A block's keys of one digit land
// side by side in the output, in key order, so inside such a run a key that
// differs from the one before starts a tile exactly and is stored as is.
// At a run's first key the key before belongs to another block: there the
// position is folded in with an atomic min, whose result the exact store,
// where a tile has one, equals.  The starts hold ~0 before the pass;
// k_ranges_finish derives the ends.
template <int ITEMS, int BITS, bool DROP, int NT, bool RANGES, typename K = uint32_t>
__global__ __launch_bounds__(NT) void k_radix_scatter(
    const K *__restrict__ kin, const uint32_t *__restrict__ vin, K *__restrict__ kout,
    uint32_t *__restrict__ vout, SegTable st, int shift, const uint32_t *__restrict__ hist_scan,
    const uint32_t *__restrict__ totals, uint32_t *__restrict__ n_kept, uint32_t ncols,
    uint32_t *__restrict__ ranges, uint32_t ntiles) {
    static_assert(!(RANGES && DROP), "ranges come from the tile sort");
    constexpr int NDIG = 1 << BITS;
    __shared__ uint32_t wcnt[(NT / 64)][NDIG];
    // gbase[d]: first the segment position of this block's first key of
    // digit d, then that minus the key's local position (staged key lp of
    // digit d goes to sbase + gbase[d] + lp)
    __shared__ uint32_t gbase[NDIG];
    constexpr int TILE = NT * ITEMS;
    constexpr int W_ITEMS = TILE / (NT / 64), W_CHUNKS = W_ITEMS / 64;
    __shared__ K skey[TILE];
    __shared__ uint32_t sval[TILE];
    __shared__ uint32_t lds_scan[(NT / 64)];
    int sg;
    uint32_t lb, sbase, n, col0, L;
    if (!xcd_block<TILE>(st, blockIdx.x, L)) return;  // idle: uniform exit
    if (!seg_block<TILE>(st, L, sg, lb, sbase, n, col0)) return;
    const uint32_t kb = st.key_base(sg);
    const size_t base = (size_t)lb * TILE;  // within the segment
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (threadIdx.x < NDIG) {
#pragma unroll
        for (int i = 0; i < (NT / 64); ++i) wcnt[i][threadIdx.x] = 0;
    }
    {
        // exclusive scan of the segment's digit totals -> digit base
        uint32_t t = threadIdx.x < NDIG ? totals[sg * RADIX + threadIdx.x] : 0u, ex;
        const uint32_t kept = block_excl_scan<uint32_t>(t, ex, lds_scan);
        if (DROP && lb == 0 && threadIdx.x == 0) n_kept[sg] = kept;
        if (threadIdx.x < NDIG)
            gbase[threadIdx.x] = ex + hist_scan[(size_t)threadIdx.x * ncols + L];
    }
    __syncthreads();

    uint32_t key[W_CHUNKS], val[W_CHUNKS], pos[W_CHUNKS];
    size_t wbase = base + (size_t)w * W_ITEMS;
#pragma unroll
    for (int c = 0; c < W_CHUNKS; ++c) {
        size_t i = wbase + (size_t)c * 64 + lane;
        bool ok = i < n;
        key[c] = ok ? kin[sbase + i] : 0u;
        val[c] = ok ? vin[sbase + i] : 0u;
    }
    // Rank of each key among the wave's keys of its digit, in input order:
    // within a chunk of 64 from the lanes below with the same digit (one
    // ballot per digit bit); across chunks from a per-wave digit counter
    // that the chunk's lowest lane of each digit advances with an LDS
    // atomic returning the count so far (the chunks' atomics run in chunk
    // order); each lane then takes its digit's base from that lowest lane.
    uint32_t lead[W_CHUNKS];
    uint32_t nloc_kept;  // keys of this block that are written
#pragma unroll
    for (int c = 0; c < W_CHUNKS; ++c) {
        size_t i = wbase + (size_t)c * 64 + lane;
        bool ok = i < n && (!DROP || key[c] != DROP_KEY);
        uint32_t d = ((key[c] - kb) >> shift) & (NDIG - 1);
        const uint64_t okm = __ballot(ok);
        uint32_t plo = (uint32_t)okm, phi = (uint32_t)(okm >> 32);
#pragma unroll
        for (int bb = 0; bb < BITS; ++bb) {
            // clear: ~0 where this lane's bit is 0, else 0.  The lanes that
            // agree with it on the bit are ballot(bit) ^ clear, so each half
            // of the update peers &= ballot(bit) ^ clear is one three-input
            // bitwise operation (truth table a & (b ^ c) = 0x60)
            uint32_t clear = (uint32_t)((int32_t)(~d << (31 - bb)) >> 31);
            asm volatile("" : "+v"(clear));  // compare this value, not a re-derived shift
            const uint64_t m = __ballot(clear == 0u);
            plo = __builtin_amdgcn_bitop3_b32(plo, (uint32_t)m, clear, (uint8_t)0x60);
            phi = __builtin_amdgcn_bitop3_b32(phi, (uint32_t)(m >> 32), clear, (uint8_t)0x60);
        }
        const uint64_t peers = (uint64_t)phi << 32 | plo;
        uint32_t rank = gs::lanes_below(peers);
        pos[c] = rank;
        lead[c] = ok ? (uint32_t)__builtin_ctzll(peers) : (uint32_t)lane;
        if (ok && rank == 0) pos[c] = atomicAdd(&wcnt[w][d], (uint32_t)__popcll(peers)) | 0x80000000u;
    }
#pragma unroll
    for (int c = 0; c < W_CHUNKS; ++c) {
        // the leader holds (count before | flag); the others their rank
        const uint32_t ld = (uint32_t)__shfl((int)pos[c], (int)lead[c], 64) & 0x7FFFFFFFu;
        pos[c] = (pos[c] & 0x80000000u) ? ld : ld + pos[c];
    }
    __syncthreads();
    {
        // per digit: the counts over the waves, the block's digit-major
        // local start, then each wave's staging base for the digit
        uint32_t d = threadIdx.x, off = 0;
        if (d < NDIG) {
#pragma unroll
            for (int i = 0; i < (NT / 64); ++i) off += wcnt[i][d];
        }
        uint32_t ex;
        nloc_kept = block_excl_scan<uint32_t>(off, ex, lds_scan);
        if (d < NDIG) {
            uint32_t run = ex;
#pragma unroll
            for (int i = 0; i < (NT / 64); ++i) {
                const uint32_t t = wcnt[i][d];
                wcnt[i][d] = run;
                run += t;
            }
            gbase[d] -= ex;
        }
    }
    __syncthreads();
    // stage in LDS in (digit, original order) order ...
#pragma unroll
    for (int c = 0; c < W_CHUNKS; ++c) {
        size_t i = wbase + (size_t)c * 64 + lane;
        if (i < n && (!DROP || key[c] != DROP_KEY)) {
            uint32_t d = ((key[c] - kb) >> shift) & (NDIG - 1);
            uint32_t lp = wcnt[w][d] + pos[c];
            skey[lp] = (K)key[c];
            sval[lp] = val[c];
        }
    }
    __syncthreads();
    // ... and write runs of equal digits to consecutive global addresses
    const uint32_t nloc = nloc_kept;
    auto put = [&](uint32_t lp, uint32_t k, uint32_t v) {
        const uint32_t d = ((k - kb) >> shift) & (NDIG - 1);
        const uint32_t dst = sbase + gbase[d] + lp;
        if (!RANGES) kout[dst] = (K)k;
        vout[dst] = v;
        if (RANGES) {
            // the key before in the block's staged order
            const uint32_t kp = lp > 0 ? skey[lp - 1] : ~0u;
            const bool first = lp == 0 || (((kp - kb) >> shift) & (NDIG - 1)) != d;
            if (k < ntiles) {  // always, for keys built here; keeps the writes in bounds
                if (first) atomicMin(&ranges[2 * k], dst);
                else if (kp != k) ranges[2 * k] = dst;
            }
        }
    };
    uint32_t lp = threadIdx.x;
    for (; lp + NT < nloc; lp += 2 * NT) {
        const uint32_t k0 = skey[lp], k1 = skey[lp + NT];
        const uint32_t v0 = sval[lp], v1 = sval[lp + NT];
        put(lp, k0, v0);
        put(lp + NT, k1, v1);
    }
    if (lp < nloc) put(lp, skey[lp], sval[lp]);
}

// Tile ends from the starts the tile sort's last pass recorded: the output
// is in tile order, so a tile ends where the next tile with keys starts, or
// at the number of sorted keys; tiles without keys (start still ~0) become
// (0, 0).  One tile per thread: the next start inside the workgroup's 256
// tiles is a suffix minimum over them (starts grow with the tile index);
// past them the workgroup looks ahead 256 tiles at a time for the first
// tile with keys.  Nothing was sorted when the splats overflowed the
// capacity.
constexpr int FINISH_THREADS = 256;
__global__ __launch_bounds__(FINISH_THREADS) void k_ranges_finish(uint32_t *__restrict__ ranges,
                                                                  uint32_t ntiles,
                                                                  const uint32_t *__restrict__ d_total,
                                                                  uint32_t cap) {
    __shared__ uint32_t sw[FINISH_THREADS / 64];
    __shared__ uint32_t s_after;
    const uint32_t N = *d_total;
    const uint32_t t = blockIdx.x * FINISH_THREADS + threadIdx.x;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint32_t st = t < ntiles ? ranges[2 * t] : ~0u;
    // inclusive suffix minimum within the wave, then over the waves above
    uint32_t m = st;
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t v = (uint32_t)__shfl_down((int)m, o, 64);
        m = lane + o < 64 ? min(m, v) : m;
    }
    if (lane == 0) sw[w] = m;
    // the first start past the workgroup's tiles
    uint32_t after = ~0u;
    for (uint32_t base = (blockIdx.x + 1) * FINISH_THREADS; base < ntiles; base += FINISH_THREADS) {
        const uint32_t i = base + threadIdx.x;
        uint32_t v = i < ntiles ? ranges[2 * i] : ~0u;
        for (int o = 32; o > 0; o >>= 1) v = min(v, (uint32_t)__shfl_xor((int)v, o, 64));
        __syncthreads();
        if (threadIdx.x == 0) s_after = ~0u;
        __syncthreads();
        if (lane == 0) atomicMin(&s_after, v);
        __syncthreads();
        after = s_after;
        if (after != ~0u) break;  // uniform
    }
    __syncthreads();
    // next start after tile t: the rest of the wave, the waves above, then past the workgroup
    uint32_t next = (uint32_t)__shfl_down((int)m, 1, 64);
    if (lane == 63) next = ~0u;
    for (int i = w + 1; i < FINISH_THREADS / 64; ++i) next = min(next, sw[i]);
    next = min(next, after);
    if (next == ~0u) next = N;
    if (t < ntiles) {
        if (st == ~0u || N > cap) {
            ranges[2 * t] = 0u;
            ranges[2 * t + 1] = 0u;
        } else {
            ranges[2 * t + 1] = next;
        }
    }
}

// Key and id buffer pairs of a sort.  The tile sort of one view with at
// most 65536 tiles carries 16-bit keys (a quarter fewer bytes per splat).
template <typename K>
struct SortBufsT {
    K *k[2];
    uint32_t *v[2];
};
using SortBufs = SortBufsT<uint32_t>;

// The scatter of a pass from buffer pair cur into cur ^ 1 (hist and totals
// already scanned).  A pass's blocks hold SORT_THREADS * ITEMS keys; the
// scatter takes each with SCATTER_THREADS threads (wider workgroups: more
// waves per CU hide the latency of its ranking and staging steps).
constexpr int SCATTER_THREADS = 512;
// (ranges: the tile sort's last pass records the tile ranges there, see
// k_radix_scatter; nullptr otherwise)
template <int ITEMS, int BITS, bool DROP, typename K>
void scatter_launch(SortBufsT<K> b, int cur, const SegTable &st, int shift, uint32_t ncols,
                    uint32_t *hist, uint32_t *totals, uint32_t *n_kept, uint32_t *ranges,
                    uint32_t ntiles, hipStream_t s) {
    constexpr int IT = ITEMS * SORT_THREADS / SCATTER_THREADS;
    static_assert(IT >= 1 && IT * SCATTER_THREADS == ITEMS * SORT_THREADS, "same block of keys");
    const dim3 grid((ncols + 7) / 8 * 8);
    if constexpr (!DROP) {
        if (ranges) {
            hipLaunchKernelGGL((k_radix_scatter<IT, BITS, false, SCATTER_THREADS, true, K>), grid,
                               dim3(SCATTER_THREADS), 0, s, b.k[cur], b.v[cur], b.k[cur ^ 1],
                               b.v[cur ^ 1], st, shift, hist, totals, n_kept, ncols, ranges, ntiles);
            return;
        }
    }
    hipLaunchKernelGGL((k_radix_scatter<IT, BITS, DROP, SCATTER_THREADS, false, K>), grid,
                       dim3(SCATTER_THREADS), 0, s, b.k[cur], b.v[cur], b.k[cur ^ 1],
                       b.v[cur ^ 1], st, shift, hist, totals, n_kept, ncols, (uint32_t *)nullptr, 0u);
}

template <int ITEMS, int BITS, bool DROP, typename K>
void radix_pass(SortBufsT<K> b, int cur, const SegTable &st, int shift, uint32_t ncols, uint32_t *hist,
                uint32_t *totals, uint32_t *n_kept, uint32_t *ranges, uint32_t ntiles,
                hipStream_t s) {
    constexpr int TILE = SORT_THREADS * ITEMS;
    constexpr int IT = TILE / SCATTER_THREADS;  // the histogram takes the same wide workgroups
    hipLaunchKernelGGL((k_radix_hist<IT, BITS, DROP, SCATTER_THREADS, K>), dim3((ncols + 7) / 8 * 8),
                       dim3(SCATTER_THREADS), 0, s, b.k[cur], st, shift, hist, ncols);
    hipLaunchKernelGGL(k_hist_rows<TILE>, dim3(1 << BITS, st.nseg), dim3(SORT_THREADS), 0, s, hist,
                       st, ncols, totals);
    scatter_launch<ITEMS, BITS, DROP>(b, cur, st, shift, ncols, hist, totals, n_kept, ranges, ntiles,
                                      s);
}

// Digit widths of a sort on `bits` key bits: ceil(bits / 8) passes of
// near-equal width (13 bits -> 7 + 6), each at least 4 bits (the keys are
// zero above `bits`, so a wider digit sorts the same).
inline int radix_passes(int bits) { return (bits + RADIX_BITS - 1) / RADIX_BITS; }
inline int radix_width(int bits, int pass) {
    int np = radix_passes(bits);
    int w = bits / np + (pass < bits % np ? 1 : 0);
    return w < 4 ? 4 : w;
}

// Sorts every segment of `st` on bits [0, bits) of (key - kbase) with
// radix_passes(bits) passes of ITEMS keys per thread; `ncols` workgroups per
// launch cover the segments' blocks.  Returns the index of the buffer pair
// holding the result.  With n_kept, the first pass drops every DROP_KEY key
// and writes how many each segment kept there; later passes sort that many.
// With p0 > 0 the first p0 passes have been done elsewhere and their result
// is in buffer pair p0 % 2.
template <int ITEMS, typename K = uint32_t>
int radix_sort(SortBufsT<K> b, SegTable st, uint32_t ncols, int bits, uint32_t *hist,
               uint32_t *totals, uint32_t *n_kept, hipStream_t s, int p0 = 0,
               uint32_t *ranges = nullptr, uint32_t ntiles = 0) {
    if (ncols == 0) ncols = 1;
    int cur = p0 & 1, shift = 0;
    for (int p = 0; p < p0; ++p) shift += radix_width(bits, p);
    for (int p = p0; p < radix_passes(bits); ++p) {
        const int w = radix_width(bits, p);
        uint32_t *rg = p + 1 == radix_passes(bits) ? ranges : nullptr;  // the last pass
        bool dropped = false;  // the depth sort's first pass (32-bit keys only)
        if constexpr (sizeof(K) == 4) {
          if (p == 0 && n_kept) {
            switch (w) {
            case 4: radix_pass<ITEMS, 4, true>(b, cur, st, shift, ncols, hist, totals, n_kept, nullptr, 0, s); break;
            case 5: radix_pass<ITEMS, 5, true>(b, cur, st, shift, ncols, hist, totals, n_kept, nullptr, 0, s); break;
            case 6: radix_pass<ITEMS, 6, true>(b, cur, st, shift, ncols, hist, totals, n_kept, nullptr, 0, s); break;
            case 7: radix_pass<ITEMS, 7, true>(b, cur, st, shift, ncols, hist, totals, n_kept, nullptr, 0, s); break;
            default: radix_pass<ITEMS, 8, true>(b, cur, st, shift, ncols, hist, totals, n_kept, nullptr, 0, s); break;
            }
            st.n_dev = n_kept;
            dropped = true;
          }
        }
        if (!dropped) {
            switch (w) {
            case 4: radix_pass<ITEMS, 4, false>(b, cur, st, shift, ncols, hist, totals, nullptr, rg, ntiles, s); break;
            case 5: radix_pass<ITEMS, 5, false>(b, cur, st, shift, ncols, hist, totals, nullptr, rg, ntiles, s); break;
            case 6: radix_pass<ITEMS, 6, false>(b, cur, st, shift, ncols, hist, totals, nullptr, rg, ntiles, s); break;
            case 7: radix_pass<ITEMS, 7, false>(b, cur, st, shift, ncols, hist, totals, nullptr, rg, ntiles, s); break;
            default: radix_pass<ITEMS, 8, false>(b, cur, st, shift, ncols, hist, totals, nullptr, rg, ntiles, s); break;
            }
        }
        shift += w;
        cur ^= 1;
    }
    return cur;
}

// Views of one bin/sort call: instance i of its V * P (Gaussian, view)
// pairs is Gaussian i % P seen from view i / P (the per-view arrays are
// view-major).  View v's tiles are numbered tbase[v] + ty * gx[v] + tx in
// the call's tile ranges.  ViewTable is the host-side description; kernels
// take a ViewRef, which holds view 0 inline (a one-view call reads nothing)
// and otherwise points at a ViewDims table the call writes to its workspace
// (small kernel arguments keep the launches of the chain cheap).
struct ViewTable {
    int nv;
    uint32_t P;
    int W[MAX_SEGS], H[MAX_SEGS];
    uint32_t gx[MAX_SEGS], tbase[MAX_SEGS];
};

struct ViewRef {
    int nv;
    uint32_t P;
    int W0, H0;
    uint32_t gx0;
    const ViewDims *vd;
    // M: a multi-view call (kernels are instantiated for both, so a
    // one-view call does no division and reads no table)
    template <bool M> __device__ __forceinline__ int view_of(uint32_t i) const { return M ? (int)(i / P) : 0; }
    template <bool M> __device__ __forceinline__ int W(int v) const { return M ? vd[v].W : W0; }
    template <bool M> __device__ __forceinline__ int H(int v) const { return M ? vd[v].H : H0; }
    template <bool M> __device__ __forceinline__ uint32_t gx(int v) const { return M ? vd[v].gx : gx0; }
    template <bool M> __device__ __forceinline__ uint32_t tbase(int v) const { return M ? vd[v].tbase : 0u; }
};

__global__ void k_put_views(ViewTable vt, ViewDims *__restrict__ out) {
    const int v = threadIdx.x;
    if (v < vt.nv) out[v] = ViewDims{vt.W[v], vt.H[v], vt.gx[v], vt.tbase[v]};
}

// ---------------------------------------------------------------------------
// Stage kernels
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t depth_key(float d) {
    uint32_t f = __float_as_uint(d);
    if (f == 0x80000000u) f = 0u;  // -0 equals +0
    return (f & 0x80000000u) ? ~f : (f | 0x80000000u);
}

__global__ void k_set_word(uint32_t *__restrict__ dst, uint32_t v) {
    if (threadIdx.x == 0) *dst = v;
}

// Precise Gaussian-tile intersection: inside the 3-sigma rectangle, keep a
// tile only if the raw opacity o exp(-q/2), q = d^T S d, reaches the 1/255
// culling threshold of Algorithm 1 somewhere in the tile's pixel box, i.e.
// the box meets the ellipse E = {d : q(d) <= T}, T = 2 (ln o + ln 255),
// S = [[a, b], [b, c]].  E is convex, so the tiles of one tile row that meet
// it are a contiguous run: the row's y-band cuts E in a convex piece whose
// x-extent is the union over its dy of the chord
//   [-b dy / a - h(dy), -b dy / a + h(dy)],
//   h(dy) = sqrt(det (ymax - |dy|) (ymax + |dy|)) / a,  ymax = sqrt(T a / det)
// (the chord's left end is convex in dy, least at the ellipse's leftmost
// point dy = b s, dx = -c s, s = sqrt(T / (c det)); the right end is
// concave, largest at dy = -b s, dx = c s), i.e. the extreme point if the
// band holds it, else the band's end chords.
// The per-Gaussian constants are FP32 (the determinant from exact FP64
// products), ymax and c s enlarged by a relative 1e-6 and T by more than
// the error of its logarithm; the per-row chord is FP32 without
// cancellation.  The band is grown by 4e-6 (ymax + |my|) + 1e-4 px (more
// than the rounding of its ends) before the chords are taken, and the run
// by 4e-6 (c s + |mx|) + 1e-4 px in x (more than the chord's rounding, every
// term of which is at most c s), so rounding can only add a boundary tile,
// never drop one.  Contraction is off so the count and emission passes agree
// bit for bit.
struct PGauss {
    float mx, my, b, inv_a;
    float det, ymax, dyl, cs;  // cs = c s = half-width of E in x; ymax = half-height
};

__device__ __forceinline__ PGauss make_pgauss(float2 m, float a, float b, float c, float lno,
                                              bool &any) {
#pragma clang fp contract(off)
    PGauss g{};
    g.mx = m.x;
    g.my = m.y;
    any = false;
    // T enlarged by more than the error of ln o (a few ulp of |ln o| <= 104,
    // from preprocess) and of this sum
    const float T = 2.0f * (lno + 5.5412635f) * (1.0f + 4e-6f) + 4e-5f;
    if (!(T >= 0.0f)) return g;  // o < 1/255: reaches the threshold nowhere
    any = true;
    const float det = (float)((double)a * (double)c - (double)b * (double)b);  // one rounding
    if (!(a > 0.0f) || !(c > 0.0f) || !(det > 0.0f)) {
        g.det = -1.0f;  // not positive definite (rounding): keep the whole rectangle
        return g;
    }
    // each value below carries a few ulp of rounding: the extents are
    // enlarged by a relative 1e-6, far beyond it
    const float s = sqrtf(T / (c * det));
    g.b = b;
    g.inv_a = 1.0f / a;
    g.det = det;
    g.ymax = sqrtf(T * a / det) * (1.0f + 1e-6f);
    g.dyl = b * s;
    g.cs = c * s * (1.0f + 1e-6f);
    return g;
}

// Columns [c0, c1] of tile row ty whose box meets E (with the margin),
// clipped to [tx0, tx1]; returns their count (0 when none).
__device__ __forceinline__ uint32_t row_span(const PGauss &g, int ty, int tx0, int tx1, int W, int H,
                                             int &c0, int &c1) {
#pragma clang fp contract(off)
    if (g.det < 0.0f) {
        c0 = tx0;
        c1 = tx1;
        return (uint32_t)(tx1 - tx0 + 1);
    }
    const float ex = 4e-6f * (g.cs + fabsf(g.mx)) + 1e-4f;
    const float ey = 4e-6f * (g.ymax + fabsf(g.my)) + 1e-4f;
    // the row's band, grown by ey, cut to the ellipse's y-extent
    const float ya = fmaxf((float)(GS_TILE * ty) - g.my - ey, -g.ymax);
    const float yb = fminf((float)min(GS_TILE * ty + GS_TILE - 1, H - 1) - g.my + ey, g.ymax);
    if (ya > yb) return 0u;
    float xl, xr;
    const float ha = sqrtf(g.det * ((g.ymax - fabsf(ya)) * (g.ymax + fabsf(ya)))) * g.inv_a;
    const float hb = sqrtf(g.det * ((g.ymax - fabsf(yb)) * (g.ymax + fabsf(yb)))) * g.inv_a;
    const float ma = -g.b * ya * g.inv_a, mb = -g.b * yb * g.inv_a;
    if (g.dyl >= ya && g.dyl <= yb) xl = -g.cs;
    else xl = fminf(ma - ha, mb - hb);
    if (-g.dyl >= ya && -g.dyl <= yb) xr = g.cs;
    else xr = fmaxf(ma + ha, mb + hb);
    const float XL = g.mx + xl - ex, XR = g.mx + xr + ex;
    // tile column c spans pixels [16c, min(16c + 15, W - 1)]
    if (XR < (float)(GS_TILE * tx0) || XL > (float)(W - 1)) return 0u;
    const float lo_f = ceilf((XL - (float)(GS_TILE - 1)) * (1.0f / GS_TILE));
    const float hi_f = floorf(XR * (1.0f / GS_TILE));
    const int lo = max((int)fmaxf(lo_f, -1.0f), tx0);
    const int hi = min((int)fminf(hi_f, 65535.0f), tx1);
    if (lo > hi) return 0u;
    c0 = lo;
    c1 = hi;
    return (uint32_t)(hi - lo + 1);
}

struct RectDec {
    int tx0, ty0, w, h;
};
__device__ __forceinline__ RectDec dec_rect(uint2 r) {
    return RectDec{(int)(r.x & 0xFFFFu), (int)(r.x >> 16), (int)(r.y & 0xFFFFu), (int)(r.y >> 16)};
}

// Depth keys and the packed tile rectangle of every Gaussian (coalesced);
// with PRECISE, a 16-byte record {rectangle, precise splat count, 0} (one
// gather for the counts kernel) and the ellipse parameters for the
// emission.  Also clears the tile ranges.  A Gaussian without splats gets
// the largest key, so it sorts after every Gaussian that has splats.
// `rects` holds uint2 rectangles, or with PRECISE uint4 records.
template <bool PRECISE, bool MULTI>
__global__ __launch_bounds__(256) void k_depth_keys(int P, const float2 *__restrict__ means2d,
                                                    const int *__restrict__ radii,
                                                    const float *__restrict__ depths,
                                                    const float *__restrict__ conics,
                                                    const float *__restrict__ lno, ViewRef vt,
                                                    uint32_t *__restrict__ keys,
                                                    uint32_t *__restrict__ ids,
                                                    void *__restrict__ rects,
                                                    PGauss *__restrict__ pg,
                                                    uint32_t *__restrict__ ranges, int n2) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    // (~0, 0) per tile for the tile sort's last pass to fold starts into;
    // (0, 0) when there are no Gaussians (no sort follows)
    if (i < n2) ranges[i] = (i & 1) || P == 0 ? 0u : ~0u;
    // (with PRECISE every lane of a wave takes part in the row loop, so
    // lanes past P stay, as Gaussians without tiles)
    if (!PRECISE && i >= P) return;
    const bool live = i < P;
    const int view = live ? vt.view_of<MULTI>((uint32_t)i) : 0;
    const int W = vt.W<MULTI>(view), H = vt.H<MULTI>(view);
    float d = live ? depths[i] : 0.0f;
    int tx0 = 0, tx1 = -1, ty0 = 0, ty1 = -1;
    int n = 0;
    float2 m = make_float2(0.f, 0.f);
    if (live && isfinite(d)) {
        m = means2d[i];
        n = gs::tile_rect(m.x, m.y, radii[i], W, H, (int)vt.gx<MULTI>(view), tx0, tx1, ty0, ty1);
    }
    uint32_t c = (uint32_t)n;
    if (PRECISE) {
        // The wave's (Gaussian, tile row) pairs are spread over its 64 lanes
        // (a Gaussian spans 1 to ~100 rows; one lane per Gaussian would make
        // the wave wait for its tallest one); each pair adds its run length
        // to its Gaussian's count in LDS.
        __shared__ PGauss s_q[256];
        __shared__ int s_rows[256][5];  // tx0, tx1, ty0 of the rectangle; W, H of the view
        __shared__ uint32_t s_start[256];
        __shared__ uint32_t s_cnt[256];
        const int lane = threadIdx.x & 63, wb = threadIdx.x & ~63;
        PGauss q{};
        uint32_t h = 0;
        if (n > 0) {
            bool any;
            q = make_pgauss(m, conics[3 * i], conics[3 * i + 1], conics[3 * i + 2],
                            lno[i - view * (int)vt.P], any);
            if (any) h = (uint32_t)(ty1 - ty0 + 1);
        }
        if (live) pg[i] = q;
        s_q[threadIdx.x] = q;
        s_rows[threadIdx.x][0] = tx0;
        s_rows[threadIdx.x][1] = tx1;
        s_rows[threadIdx.x][2] = ty0;
        s_rows[threadIdx.x][3] = W;
        s_rows[threadIdx.x][4] = H;
        s_cnt[threadIdx.x] = 0u;
        // exclusive prefix of h over the wave
        uint32_t incl = h;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const uint32_t o = __shfl_up(incl, d, 64);
            if (lane >= d) incl += o;
        }
        s_start[threadIdx.x] = incl - h;
        const uint32_t total = __shfl(incl, 63, 64);
        __builtin_amdgcn_wave_barrier();  // the wave's LDS entries are written
        for (uint32_t p0 = 0; p0 < total; p0 += 64) {
            const uint32_t p = p0 + (uint32_t)lane;
            if (p < total) {
                uint32_t lo = 0, hi = 64;  // last lane whose first pair is <= p
                while (hi - lo > 1) {
                    const uint32_t mid = (lo + hi) >> 1;
                    if (s_start[wb + mid] <= p) lo = mid;
                    else hi = mid;
                }
                const int o = wb + (int)lo;
                int c0, c1;
                const uint32_t r = row_span(s_q[o], s_rows[o][2] + (int)(p - s_start[o]),
                                            s_rows[o][0], s_rows[o][1], s_rows[o][3],
                                            s_rows[o][4], c0, c1);
                if (r) atomicAdd(&s_cnt[o], r);
            }
        }
        // LDS operations of a wave complete in order: the sums are final
        __builtin_amdgcn_wave_barrier();
        c = s_cnt[threadIdx.x];
        if (!live) return;
    }
    keys[i] = c > 0 ? depth_key(d) : 0xFFFFFFFFu;
    ids[i] = (uint32_t)i;
    const uint2 r = c > 0 ? make_uint2((uint32_t)tx0 | ((uint32_t)ty0 << 16),
                                       (uint32_t)(tx1 - tx0 + 1) | ((uint32_t)(ty1 - ty0 + 1) << 16))
                          : make_uint2(0u, 0u);
    if (PRECISE)
        ((uint4 *)rects)[i] = make_uint4(r.x, r.y, c, 0u);
    else
        ((uint2 *)rects)[i] = r;
}

// Rectangle and splat count of each instance in depth order (view by view;
// zero past the n_vis[v] instances of view v that have splats), and each
// block's sum of counts.
template <bool PRECISE, bool MULTI>
__global__ __launch_bounds__(COUNT_THREADS) void k_counts(int P, const uint32_t *__restrict__ order,
                                                         const void *__restrict__ rects,
                                                         uint2 *__restrict__ rects_sorted,
                                                         uint32_t *__restrict__ cnt,
                                                         const uint32_t *__restrict__ n_vis,
                                                         uint64_t *__restrict__ part, ViewRef vt) {
    __shared__ uint64_t lds[COUNT_THREADS / 64];
    const size_t base = (size_t)blockIdx.x * SORT_TILE;
    uint64_t sum = 0;
    const uint32_t nvis0 = n_vis[0];
    // two rounds of loads for all the thread's items (the order entries,
    // then the rectangles they name) rather than two dependent loads per
    // item.  Slots past a view's Gaussians with splats (and past the end:
    // the index is clamped, P >= 1 here) hold no valid id and read
    // Gaussian 0 instead; their outputs are zero.
    uint32_t g[SORT_ITEMS];
    bool has[SORT_ITEMS];
#pragma unroll
    for (int k = 0; k < SORT_ITEMS; ++k) {
        const size_t j = base + (size_t)k * COUNT_THREADS + threadIdx.x;
        const size_t jc = j < (size_t)P ? j : (size_t)P - 1;
        const int v = vt.view_of<MULTI>((uint32_t)jc);
        has[k] = j < (size_t)P && jc - (size_t)v * vt.P < (MULTI ? n_vis[v] : nvis0);
        const uint32_t o = order[jc];
        g[k] = has[k] ? o : 0u;
    }
    uint2 r[SORT_ITEMS];
    uint32_t cg[SORT_ITEMS];
#pragma unroll
    for (int k = 0; k < SORT_ITEMS; ++k) {
        if (PRECISE) {
            const uint4 q = ((const uint4 *)rects)[g[k]];
            r[k] = make_uint2(q.x, q.y);
            cg[k] = q.z;
        } else {
            r[k] = ((const uint2 *)rects)[g[k]];
            cg[k] = 0u;
        }
    }
#pragma unroll
    for (int k = 0; k < SORT_ITEMS; ++k) {
        const size_t j = base + (size_t)k * COUNT_THREADS + threadIdx.x;
        if (j < (size_t)P) {
            const uint2 rr = has[k] ? r[k] : make_uint2(0u, 0u);
            const uint32_t c = !has[k] ? 0u : PRECISE ? cg[k] : (rr.y & 0xFFFFu) * (rr.y >> 16);
            rects_sorted[j] = rr;
            cnt[j] = c;
            sum += c;
        }
    }
    uint64_t ex;
    const uint64_t tot = block_excl_scan<uint64_t>(sum, ex, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// Stages the Gaussians of output window `blk` (slots [blk * WIN, +WIN)):
// those with splats among j0 = owner of its first slot up to j1 = owner of
// the next window's first slot (or of the last slot).  Within one view
// every instance in between owns at least one slot of the window; across a
// view boundary the instances of view v without splats (positions
// [v P + n_vis[v], (v + 1) P)) are skipped.  So at most WIN + 1 are staged.
// Returns their number m, or 0 when the window is idle (overflow, past N).
// All threads of the block call it.
template <int WIN, int NT, bool MULTI>
__device__ __forceinline__ uint32_t stage_window(int P, const uint32_t *__restrict__ order,
                                                 const uint32_t *__restrict__ offs,
                                                 const uint2 *__restrict__ rects_sorted,
                                                 const uint32_t *__restrict__ win_start,
                                                 uint32_t nwin, uint32_t N, uint32_t cap,
                                                 const ViewRef &vt,
                                                 const uint32_t *__restrict__ n_vis,
                                                 uint32_t *s_off, uint2 *s_rect, uint32_t *s_id) {
    const uint32_t o0 = blockIdx.x * (uint32_t)WIN;
    if (N > cap || o0 >= N || blockIdx.x + 1 >= nwin) return 0u;
    const uint32_t j0 = win_start[blockIdx.x];
    const uint32_t j1 = win_start[blockIdx.x + 1];
    if (j0 >= (uint32_t)P || j1 >= (uint32_t)P || j1 < j0) return 0u;  // cannot happen when the scan ran
    if (!MULTI) {  // one view: every instance in [j0, j1] owns a slot
        const uint32_t m = min(j1 - j0 + 1u, (uint32_t)WIN + 1u);
        for (uint32_t k = threadIdx.x; k < m; k += NT) {
            s_off[k] = offs[j0 + k];
            s_rect[k] = rects_sorted[j0 + k];
            s_id[k] = order[j0 + k];
        }
        return m;
    }
    const int v0 = vt.view_of<MULTI>(j0), v1 = vt.view_of<MULTI>(j1);
    uint32_t m = 0;
    for (int v = v0; v <= v1 && m < (uint32_t)WIN + 1u; ++v) {
        // view v's instances with splats that lie in [j0, j1]
        const uint32_t vb = (uint32_t)v * vt.P;
        const uint32_t lo = max(j0, vb), hi = min(j1 + 1u, vb + n_vis[v]);
        if (hi <= lo) continue;
        const uint32_t len = min(hi - lo, (uint32_t)WIN + 1u - m);
        for (uint32_t k = threadIdx.x; k < len; k += NT) {
            s_off[m + k] = offs[lo + k];
            s_rect[m + k] = rects_sorted[lo + k];
            s_id[m + k] = order[lo + k];
        }
        m += len;
    }
    return m;
}

// Largest i in [0, n) with a[i] <= x (a non-decreasing, a[0] <= x).
__device__ __forceinline__ uint32_t last_le(const uint32_t *a, uint32_t n, uint32_t x) {
    uint32_t lo = 0, hi = n;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (a[mid] <= x) lo = mid;
        else hi = mid;
    }
    return lo;
}

// The EMIT_ITEMS consecutive slots from s0 (< oend) of a staged window under
// the 3-sigma rule: the owner of s0 by binary search, then the rectangles
// walked in row-major order; written from registers with one 16-byte store
// per array (consecutive threads, consecutive 16-byte pieces).  With HIST,
// each key's lowest digit (key & dmask) is also counted in hcount (LDS).
template <bool MULTI, bool HIST, typename K, int IT = EMIT_ITEMS>
__device__ __forceinline__ void emit_slots(uint32_t s0, uint32_t oend, const uint32_t *s_off,
                                           const uint2 *s_rect, const uint32_t *s_id, uint32_t m,
                                           const ViewRef &vt, K *__restrict__ tkey,
                                           uint32_t *__restrict__ tid, uint32_t dmask,
                                           uint32_t *hcount) {
    static_assert(IT == 4 || IT == 8, "whole 16-byte stores");
    uint32_t tk[IT], tg[IT];
    {
        uint32_t k = last_le(s_off, m, s0);
        const uint32_t l = s0 - s_off[k];
        uint2 r = s_rect[k];
        uint32_t w = max(r.y & 0xFFFFu, 1u), h = max(r.y >> 16, 1u);
        uint32_t row = l / w, col = l - row * w;
        // the Gaussian's view: its tile numbering and its id within the view
        int v = vt.view_of<MULTI>(s_id[k]);
        uint32_t gid = s_id[k] - (uint32_t)v * vt.P;
#pragma unroll
        for (int i = 0; i < IT; ++i) {
            const uint32_t tx = (r.x & 0xFFFFu) + col, ty = (r.x >> 16) + row;
            tk[i] = vt.tbase<MULTI>(v) + ty * vt.gx<MULTI>(v) + tx;
            tg[i] = gid;
            if (++col == w) {
                col = 0;
                if (++row == h && k + 1 < m) {
                    row = 0;
                    ++k;
                    r = s_rect[k];
                    w = max(r.y & 0xFFFFu, 1u);
                    h = max(r.y >> 16, 1u);
                    v = vt.view_of<MULTI>(s_id[k]);
                    gid = s_id[k] - (uint32_t)v * vt.P;
                }
            }
        }
    }
    const bool vec = s0 + IT <= oend && gs::aligned(tkey + s0, IT * sizeof(K)) &&
                     gs::aligned(tid + s0, 16);
    if (vec) {
        if constexpr (sizeof(K) == 4) {
#pragma unroll
            for (int i = 0; i < IT; i += 4)
                *(uint4 *)(tkey + s0 + i) = make_uint4(tk[i], tk[i + 1], tk[i + 2], tk[i + 3]);
        } else if constexpr (IT == 4) {  // four 16-bit keys in one 8-byte store
            *(uint2 *)(tkey + s0) = make_uint2(tk[0] | tk[1] << 16, tk[2] | tk[3] << 16);
        } else {  // eight in one 16-byte store
            *(uint4 *)(tkey + s0) = make_uint4(tk[0] | tk[1] << 16, tk[2] | tk[3] << 16,
                                               tk[4] | tk[5] << 16, tk[6] | tk[7] << 16);
        }
#pragma unroll
        for (int i = 0; i < IT; i += 4)
            *(uint4 *)(tid + s0 + i) = make_uint4(tg[i], tg[i + 1], tg[i + 2], tg[i + 3]);
    } else {
#pragma unroll
        for (int i = 0; i < IT; ++i) {
            if (s0 + (uint32_t)i < oend) {
                tkey[s0 + i] = (K)tk[i];
                tid[s0 + i] = tg[i];
            }
        }
    }
    if (HIST) {
#pragma unroll
        for (int i = 0; i < IT; ++i)
            if (s0 + (uint32_t)i < oend) atomicAdd(&hcount[tk[i] & dmask], 1u);
    }
}

// Expands the splats of output window blockIdx.x (EMIT_TILE consecutive
// slots) under the 3-sigma rule, EMIT_ITEMS slots per thread.
//
// With HIST (one view), the window also counts its keys' lowest digit (key &
// dmask, at most RADIX digits) for the first tile pass and writes the counts
// to hist2[window * RADIX + d], so that pass needs no histogram kernel of its
// own; windows past the splats write nothing.
template <bool MULTI, bool HIST, typename K = uint32_t>
__global__ __launch_bounds__(EMIT_THREADS) void k_emit(int P, const uint32_t *__restrict__ order,
                                                       const uint32_t *__restrict__ offs,
                                                       const uint2 *__restrict__ rects_sorted,
                                                       const uint32_t *__restrict__ win_start,
                                                       uint32_t nwin, ViewRef vt,
                                                       const uint32_t *__restrict__ n_vis,
                                                       const uint32_t *__restrict__ n_splats,
                                                       uint32_t cap, K *__restrict__ tkey,
                                                       uint32_t *__restrict__ tid, uint32_t dmask,
                                                       uint32_t *__restrict__ hist2) {
    static_assert(EMIT_ITEMS == 4, "one 16-byte store per thread and array");
    static_assert(EMIT_THREADS > RADIX, "one thread per digit count");
    static_assert(!(MULTI && HIST), "the windows of a multi-view call cross views");
    __shared__ uint32_t s_off[EMIT_TILE + 1];
    __shared__ uint2 s_rect[EMIT_TILE + 1];
    __shared__ uint32_t s_id[EMIT_TILE + 1];
    __shared__ uint32_t hcount[HIST ? RADIX : 1];
    const uint32_t N = *n_splats;
    const uint32_t m = stage_window<EMIT_TILE, EMIT_THREADS, MULTI>(P, order, offs, rects_sorted, win_start,
                                                             nwin, N, cap, vt, n_vis, s_off,
                                                             s_rect, s_id);
    if (m == 0) return;  // block-uniform
    if (HIST && threadIdx.x <= dmask) hcount[threadIdx.x] = 0u;
    __syncthreads();
    const uint32_t o0 = blockIdx.x * (uint32_t)EMIT_TILE;
    const uint32_t oend = min(o0 + (uint32_t)EMIT_TILE, N);
    const uint32_t s0 = o0 + (uint32_t)threadIdx.x * EMIT_ITEMS;
    if (s0 < oend)
        emit_slots<MULTI, HIST, K>(s0, oend, s_off, s_rect, s_id, m, vt, tkey, tid, dmask, hcount);
    if (HIST) {
        __syncthreads();
        if (threadIdx.x <= dmask)  // one contiguous row of counts per window
            hist2[(size_t)blockIdx.x * RADIX + threadIdx.x] = hcount[threadIdx.x];
    }
}

// One view, 3-sigma rule: window blockIdx.x (EMIT_TILE slots) with 256
// threads of 8 slots, so twice as many windows fit on a CU as with k_emit
// (one window is a chain of dependent steps: staging loads, search, walk,
// stores).  Up to EMIT1_CAP + 1 Gaussians are staged in LDS (16 KB); a
// window with more (its Gaussians average under two slots) searches and
// walks the global arrays instead.  HIST as for k_emit.
constexpr int EMIT1_THREADS = 256;
constexpr int EMIT1_ITEMS = EMIT_TILE / EMIT1_THREADS;
constexpr uint32_t EMIT1_CAP = 1024;
template <bool HIST, typename K>
__global__ __launch_bounds__(EMIT1_THREADS) void k_emit1(int P, const uint32_t *__restrict__ order,
                                                         const uint32_t *__restrict__ offs,
                                                         const uint2 *__restrict__ rects_sorted,
                                                         const uint32_t *__restrict__ win_start,
                                                         uint32_t nwin, ViewRef vt,
                                                         const uint32_t *__restrict__ n_splats,
                                                         uint32_t cap, K *__restrict__ tkey,
                                                         uint32_t *__restrict__ tid, uint32_t dmask,
                                                         uint32_t *__restrict__ hist2) {
    static_assert(EMIT1_THREADS >= RADIX, "one thread per digit count");
    __shared__ uint32_t s_off[EMIT1_CAP + 1];
    __shared__ uint2 s_rect[EMIT1_CAP + 1];
    __shared__ uint32_t s_id[EMIT1_CAP + 1];
    __shared__ uint32_t hcount[HIST ? RADIX : 1];
    const uint32_t N = *n_splats;
    const uint32_t o0 = blockIdx.x * (uint32_t)EMIT_TILE;
    if (N > cap || o0 >= N || blockIdx.x + 1 >= nwin) return;  // block-uniform
    const uint32_t j0 = win_start[blockIdx.x];
    const uint32_t j1 = win_start[blockIdx.x + 1];
    if (j0 >= (uint32_t)P || j1 >= (uint32_t)P || j1 < j0) return;  // cannot happen when the scan ran
    // every instance in [j0, j1] owns a slot (one view)
    const uint32_t m = j1 - j0 + 1u;
    const bool staged = m <= EMIT1_CAP + 1u;
    if (staged) {
        for (uint32_t k = threadIdx.x; k < m; k += EMIT1_THREADS) {
            s_off[k] = offs[j0 + k];
            s_rect[k] = rects_sorted[j0 + k];
            s_id[k] = order[j0 + k];
        }
    }
    if (HIST && threadIdx.x <= dmask) hcount[threadIdx.x] = 0u;
    __syncthreads();
    const uint32_t oend = min(o0 + (uint32_t)EMIT_TILE, N);
    const uint32_t s0 = o0 + (uint32_t)threadIdx.x * EMIT1_ITEMS;
    if (s0 < oend) {
        if (staged)
            emit_slots<false, HIST, K, EMIT1_ITEMS>(s0, oend, s_off, s_rect, s_id, m, vt, tkey, tid,
                                                    dmask, hcount);
        else
            emit_slots<false, HIST, K, EMIT1_ITEMS>(s0, oend, offs + j0, rects_sorted + j0,
                                                    order + j0, m, vt, tkey, tid, dmask, hcount);
    }
    if (HIST) {
        __syncthreads();
        if (threadIdx.x <= dmask)  // one contiguous row of counts per window
            hist2[(size_t)blockIdx.x * RADIX + threadIdx.x] = hcount[threadIdx.x];
    }
}

// The first tile pass's digit counts per block of BLK keys, from the counts
// k_emit<false, true> wrote per emission window of WIN slots (one row of
// RADIX counts per window): a block's counts are the sum of its G = BLK /
// WIN windows' rows.  Workgroup j takes blocks 16 j .. 16 j + 15: thread d
// reads digit d of each window (the rows are read whole, 256 threads at a
// time; threads past the pass's digits idle) and writes digit d's 16 block counts side by side into
// hist[d * ncols + block], the layout the row scan (k_hist_rows) and the
// scatter read.  One segment (one view).
constexpr int WIN_BLOCKS = 16;
template <int WIN, int BLK>
__global__ __launch_bounds__(SORT_THREADS) void k_windows_to_blocks(const uint32_t *__restrict__ hist2,
                                                                    SegTable st, uint32_t ncols,
                                                                    uint32_t ndig,
                                                                    uint32_t *__restrict__ hist) {
    constexpr uint32_t G = BLK / WIN;
    static_assert(BLK % WIN == 0 && RADIX == SORT_THREADS, "whole windows; one digit per thread");
    uint32_t base, n;
    st.get(0, base, n);
    const uint32_t nb = (n + BLK - 1u) / BLK, nw = (n + WIN - 1u) / WIN;
    const uint32_t b0 = blockIdx.x * WIN_BLOCKS;
    if (b0 >= nb) return;  // uniform
    const uint32_t d = threadIdx.x;
    if (d >= ndig) return;  // digits the pass does not use (whole waves)
    uint32_t v[WIN_BLOCKS];
#pragma unroll
    for (int i = 0; i < WIN_BLOCKS; ++i) {
        uint32_t acc = 0u;
#pragma unroll
        for (uint32_t g = 0; g < G; ++g) {
            const uint32_t w = (b0 + i) * G + g;
            const uint32_t x = hist2[(size_t)(w < nw ? w : nw - 1u) * RADIX + d];
            acc += w < nw ? x : 0u;
        }
        v[i] = acc;
    }
#pragma unroll
    for (int i = 0; i < WIN_BLOCKS; ++i)
        if (b0 + i < nb) hist[(size_t)d * ncols + b0 + i] = v[i];
}

// Exclusive prefix sum of a[0, n) in place (n <= NT * 8); returns the total.
// All threads of the block call it; `lds` holds NT / 64 entries.
template <int NT>
__device__ __forceinline__ uint32_t block_scan_array(uint32_t *a, uint32_t n, uint32_t *lds) {
    const uint32_t per = (n + NT - 1) / NT;
    const uint32_t b = threadIdx.x * per, e = min(b + per, n);
    uint32_t sum = 0;
    for (uint32_t i = b; i < e; ++i) sum += a[i];
    uint32_t ex;
    const uint32_t tot = block_excl_scan<uint32_t>(sum, ex, lds);
    for (uint32_t i = b; i < e; ++i) {
        const uint32_t v = a[i];
        a[i] = ex;
        ex += v;
    }
    __syncthreads();
    return tot;
}

// Precise rule: expands window blockIdx.x (EMIT_TILE_P slots).  The window's
// Gaussians' tile rows are listed as (Gaussian, row) pairs; each pair's run
// of tiles [c0, c0 + n) is computed once (one row_span per pair, spread over
// the block), the runs' first slots come from a prefix sum over n, and every
// thread then finds the run holding its first slot by binary search and
// writes its EMIT_ITEMS_P tiles directly.  A window with more than RCAP
// pairs (several very tall Gaussians) walks the rows per thread instead.
template <bool MULTI, typename K = uint32_t>
__global__ __launch_bounds__(EMIT_THREADS_P) void k_emit_precise(
    int P, const uint32_t *__restrict__ order, const uint32_t *__restrict__ offs,
    const uint2 *__restrict__ rects_sorted, const PGauss *__restrict__ pg,
    const uint32_t *__restrict__ win_start, uint32_t nwin, ViewRef vt,
    const uint32_t *__restrict__ n_vis, const uint32_t *__restrict__ n_splats, uint32_t cap,
    K *__restrict__ tkey,
    uint32_t *__restrict__ tid) {
    constexpr int WIN = EMIT_TILE_P;
    __shared__ uint32_t s_off[WIN + 1];
    __shared__ uint2 s_rect[WIN + 1];
    __shared__ uint32_t s_id[WIN + 1];
    __shared__ uint32_t s_hoff[WIN + 1];   // first pair of each Gaussian
    __shared__ uint32_t s_pslot[RCAP];     // first slot of each pair's run
    __shared__ uint16_t s_pk[RCAP], s_pty[RCAP], s_pc0[RCAP], s_pn[RCAP];
    __shared__ uint32_t s_tk[WIN];
    __shared__ uint32_t s_tg[WIN];
    __shared__ uint32_t s_scan[EMIT_THREADS_P / 64];
    const uint32_t N = *n_splats;
    const uint32_t m = stage_window<WIN, EMIT_THREADS_P, MULTI>(P, order, offs, rects_sorted, win_start,
                                                       nwin, N, cap, vt, n_vis, s_off, s_rect,
                                                       s_id);
    if (m == 0) return;  // block-uniform
    __syncthreads();
    const uint32_t o0 = blockIdx.x * (uint32_t)WIN;
    const uint32_t oend = min(o0 + (uint32_t)WIN, N);
    const uint32_t s0 = o0 + (uint32_t)threadIdx.x * EMIT_ITEMS_P;
    // placeholders (tile 0, Gaussian 0: in bounds) for slots a disagreement
    // between the count and this pass would leave unwritten
    for (int i = 0; i < EMIT_ITEMS_P && s0 + (uint32_t)i < oend; ++i) {
        s_tk[s0 + i - o0] = 0u;
        s_tg[s0 + i - o0] = 0u;
    }
    for (uint32_t k = threadIdx.x; k < m; k += EMIT_THREADS_P) s_hoff[k] = s_rect[k].y >> 16;
    __syncthreads();
    const uint32_t R = block_scan_array<EMIT_THREADS_P>(s_hoff, m, s_scan);
    if (R <= (uint32_t)RCAP) {
        for (uint32_t p = threadIdx.x; p < R; p += EMIT_THREADS_P) {
            const uint32_t k = last_le(s_hoff, m, p);
            const RectDec d = dec_rect(s_rect[k]);
            const int ty = d.ty0 + (int)(p - s_hoff[k]);
            const PGauss q = pg[s_id[k]];
            const int v = vt.view_of<MULTI>(s_id[k]);
            int c0 = 0, c1 = -1;
            const uint32_t n = row_span(q, ty, d.tx0, d.tx0 + d.w - 1, vt.W<MULTI>(v), vt.H<MULTI>(v), c0, c1);
            s_pk[p] = (uint16_t)k;
            s_pty[p] = (uint16_t)ty;
            s_pc0[p] = (uint16_t)c0;
            s_pn[p] = (uint16_t)n;
            s_pslot[p] = n;
        }
        __syncthreads();
        block_scan_array<EMIT_THREADS_P>(s_pslot, R, s_scan);
        // absolute first slots: Gaussian k's first run starts at s_off[k]
        for (uint32_t k = threadIdx.x; k < m; k += EMIT_THREADS_P)
            s_hoff[k] = s_off[k] - s_pslot[s_hoff[k]];
        __syncthreads();
        for (uint32_t p = threadIdx.x; p < R; p += EMIT_THREADS_P) s_pslot[p] += s_hoff[s_pk[p]];
        __syncthreads();
        if (s0 < oend) {
            // the last run starting at or before s0 is non-empty and holds it
            uint32_t p = last_le(s_pslot, R, s0);
            uint32_t within = s0 - s_pslot[p];
            for (int i = 0; i < EMIT_ITEMS_P; ++i) {
                const uint32_t o = s0 + (uint32_t)i;
                if (o >= oend || within >= s_pn[p]) break;
                const uint32_t g = s_id[s_pk[p]];
                const int v = vt.view_of<MULTI>(g);
                s_tk[o - o0] = vt.tbase<MULTI>(v) + (uint32_t)s_pty[p] * vt.gx<MULTI>(v) + s_pc0[p] + within;
                s_tg[o - o0] = g - (uint32_t)v * vt.P;
                if (++within < s_pn[p]) continue;
                within = 0;
                do {
                    ++p;
                } while (p < R && s_pn[p] == 0);
                if (p >= R) break;
            }
        }
    } else if (s0 < oend) {
        // per-thread walk along the rows
        uint32_t k = last_le(s_off, m, s0);
        uint32_t l = s0 - s_off[k];
        PGauss q = pg[s_id[k]];
        RectDec d = dec_rect(s_rect[k]);
        int v = vt.view_of<MULTI>(s_id[k]);
        int W = vt.W<MULTI>(v), H = vt.H<MULTI>(v);
        int ty = d.ty0, c0 = 0, c1 = -1;
        uint32_t n = row_span(q, ty, d.tx0, d.tx0 + d.w - 1, W, H, c0, c1);
        while (l >= n && ty < d.ty0 + d.h - 1) {  // row holding local slot l
            l -= n;
            ++ty;
            n = row_span(q, ty, d.tx0, d.tx0 + d.w - 1, W, H, c0, c1);
        }
        for (int i = 0; i < EMIT_ITEMS_P; ++i) {
            const uint32_t o = s0 + (uint32_t)i;
            if (o >= oend || l >= n) break;  // (l >= n only if the counts disagree)
            s_tk[o - o0] = vt.tbase<MULTI>(v) + (uint32_t)ty * vt.gx<MULTI>(v) + (uint32_t)(c0 + (int)l);
            s_tg[o - o0] = s_id[k] - (uint32_t)v * vt.P;
            if (++l < n) continue;
            l = 0;
            n = 0;
            while (n == 0 && ty < d.ty0 + d.h - 1) {  // next row with tiles
                ++ty;
                n = row_span(q, ty, d.tx0, d.tx0 + d.w - 1, W, H, c0, c1);
            }
            if (n > 0) continue;
            ++k;  // next Gaussian (each one in the window has a slot)
            if (k >= m) break;
            q = pg[s_id[k]];
            d = dec_rect(s_rect[k]);
            v = vt.view_of<MULTI>(s_id[k]);
            W = vt.W<MULTI>(v);
            H = vt.H<MULTI>(v);
            ty = d.ty0;
            n = row_span(q, ty, d.tx0, d.tx0 + d.w - 1, W, H, c0, c1);
            while (n == 0 && ty < d.ty0 + d.h - 1) {
                ++ty;
                n = row_span(q, ty, d.tx0, d.tx0 + d.w - 1, W, H, c0, c1);
            }
        }
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < oend - o0; i += EMIT_THREADS_P) {
        tkey[o0 + i] = (K)s_tk[i];
        tid[o0 + i] = s_tg[i];
    }
}

// Workspace carve-up (every region 256-byte aligned) for n = V * P
// instances and room for `cap` splats.
struct Layout {
    size_t dkey0, dkey1, did0, did1, rects, rects_sorted, cnt, offs, pg, tkey0, tkey1, tid,
        hist, totals, nvis, bounds, vdims, part, win, total;
    uint32_t nwin, ncols_depth, ncols_tile;
};

// Keys per thread of the tile sort's blocks.
inline int tile_items(uint32_t nv, uint32_t cap) {
    return nv == 1 && cap >= BIG_SORT_CAP ? TILE_ITEMS_BIG : TILE_ITEMS;
}

Layout layout(uint32_t nv, uint32_t P, uint32_t cap, bool precise) {
    Layout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align_up(off + (bytes ? bytes : 4), 256);
        return o;
    };
    const size_t n = (size_t)nv * P;
    L.ncols_depth = nv * ((P + SORT_THREADS * DEPTH_ITEMS - 1) / (SORT_THREADS * DEPTH_ITEMS));
    const uint32_t tblk = SORT_THREADS * tile_items(nv, cap);
    L.ncols_tile = (cap + tblk - 1) / tblk + nv;
    const uint32_t ncols = L.ncols_depth > L.ncols_tile ? L.ncols_depth : L.ncols_tile;
    const uint32_t win = precise ? EMIT_TILE_P : EMIT_TILE;
    L.nwin = (cap + win - 1) / win + 2;
    L.dkey0 = take(4 * n);
    L.dkey1 = take(4 * n);
    L.did0 = take(4 * n);
    L.did1 = take(4 * n);
    L.rects = take((precise ? 16 : 8) * n);  // uint2 rectangles, or {rectangle, count} records
    L.rects_sorted = take(8 * n);
    L.cnt = take(4 * n);
    L.offs = take(4 * n);
    L.pg = take(precise ? sizeof(PGauss) * n : 0);
    L.tkey0 = take(4ull * cap);
    L.tkey1 = take(4ull * cap);
    L.tid = take(4ull * cap);
    L.hist = take(4ull * RADIX * ncols);
    L.totals = take(4ull * RADIX * nv);
    L.nvis = take(4ull * nv);
    L.bounds = take(4ull * (nv + 1));
    L.vdims = take(sizeof(ViewDims) * nv);
    L.part = take(8 * ((n + SORT_TILE - 1) / SORT_TILE + 2));
    L.win = take(4ull * L.nwin);
    L.total = off;
    return L;
}

int ceil_log2(uint32_t x) {
    int b = 0;
    while ((1ull << b) < x) ++b;
    return b;
}

// Per-view image sizes -> the view table, the total tile count and the
// widest per-view tile index (bits); false for invalid sizes.
bool make_views(int nv, uint32_t P, const int32_t *widths, const int32_t *heights, ViewTable &vt,
                uint32_t &ntiles, int &tbits) {
    if (nv < 1 || nv > GS_MAX_BIN_VIEWS || !widths || !heights) return false;
    vt = ViewTable{};
    vt.nv = nv;
    vt.P = P;
    uint64_t acc = 0;
    tbits = 1;
    for (int v = 0; v < nv; ++v) {
        const int w = widths[v], h = heights[v];
        if (w <= 0 || h <= 0 || w > GS_MAX_DIM || h > GS_MAX_DIM) return false;
        const uint32_t gx = (uint32_t)gs::grid_x(w), nt = gx * (uint32_t)gs::grid_y(h);
        vt.W[v] = w;
        vt.H[v] = h;
        vt.gx[v] = gx;
        vt.tbase[v] = (uint32_t)acc;
        acc += nt;
        const int b = ceil_log2(nt);
        if (b > tbits) tbits = b;
    }
    if (acc >= 0x40000000ull) return false;
    ntiles = (uint32_t)acc;
    return true;
}

// Splats of each view (bounds[v + 1] - bounds[v]).
__global__ void k_view_splats(const uint32_t *__restrict__ bounds, int nv,
                              uint32_t *__restrict__ out) {
    const int v = threadIdx.x;
    if (v < nv) out[v] = bounds ? bounds[v + 1] - bounds[v] : 0u;
}

}  // namespace

extern "C" size_t gs_bin_sort_workspace_bytes(int32_t P, uint32_t capacity, int32_t width,
                                              int32_t height) {
    if (P < 0 || width <= 0 || height <= 0 || width > GS_MAX_DIM || height > GS_MAX_DIM) return 0;
    if (capacity >= 0x80000000u) return 0;
    return layout(1, (uint32_t)P, capacity, false).total;
}

extern "C" size_t gs_bin_sort_precise_workspace_bytes(int32_t P, uint32_t capacity, int32_t width,
                                                      int32_t height) {
    if (P < 0 || width <= 0 || height <= 0 || width > GS_MAX_DIM || height > GS_MAX_DIM) return 0;
    if (capacity >= 0x80000000u) return 0;
    return layout(1, (uint32_t)P, capacity, true).total;
}

extern "C" size_t gs_bin_sort_multiview_workspace_bytes(int32_t nviews, int32_t P,
                                                        uint32_t capacity, const int32_t *widths,
                                                        const int32_t *heights, int32_t precise) {
    ViewTable vt;
    uint32_t ntiles;
    int tbits;
    if (P < 0 || capacity >= 0x80000000u) return 0;
    if (!make_views(nviews, (uint32_t)P, widths, heights, vt, ntiles, tbits)) return 0;
    if ((uint64_t)nviews * (uint64_t)P >= 0x80000000ull) return 0;
    return layout((uint32_t)nviews, (uint32_t)P, capacity, precise != 0).total;
}

namespace {

// The tile sort of a call, ITEMS keys per thread.  With emit_hist, the
// expansion has counted the first pass's digits per window into hist2: the
// pass then only scans and scatters.  Returns the buffer pair holding the
// result.
template <int ITEMS, typename K>
int tile_sort(SortBufsT<K> tb, const SegTable &st, uint32_t ncols, int tbits, bool emit_hist,
              const uint32_t *hist2, uint32_t *hist, uint32_t *totals, uint32_t *ranges,
              uint32_t ntiles, hipStream_t s) {
    if (emit_hist) {
        const int w0 = radix_width(tbits, 0);
        uint32_t *rg = radix_passes(tbits) == 1 ? ranges : nullptr;  // a one-pass sort
        hipLaunchKernelGGL((k_windows_to_blocks<EMIT_TILE, SORT_THREADS * ITEMS>),
                           dim3((ncols + WIN_BLOCKS - 1) / WIN_BLOCKS), dim3(SORT_THREADS), 0, s,
                           hist2, st, ncols, 1u << w0, hist);
        hipLaunchKernelGGL(k_hist_rows<SORT_THREADS * ITEMS>, dim3(1 << w0, 1), dim3(SORT_THREADS),
                           0, s, hist, st, ncols, totals);
        switch (w0) {
        case 4: scatter_launch<ITEMS, 4, false>(tb, 0, st, 0, ncols, hist, totals, nullptr, rg, ntiles, s); break;
        case 5: scatter_launch<ITEMS, 5, false>(tb, 0, st, 0, ncols, hist, totals, nullptr, rg, ntiles, s); break;
        case 6: scatter_launch<ITEMS, 6, false>(tb, 0, st, 0, ncols, hist, totals, nullptr, rg, ntiles, s); break;
        case 7: scatter_launch<ITEMS, 7, false>(tb, 0, st, 0, ncols, hist, totals, nullptr, rg, ntiles, s); break;
        default: scatter_launch<ITEMS, 8, false>(tb, 0, st, 0, ncols, hist, totals, nullptr, rg, ntiles, s); break;
        }
    }
    return radix_sort<ITEMS, K>(tb, st, ncols, tbits, hist, totals, nullptr, s, emit_hist ? 1 : 0,
                                ranges, ntiles);
}

gs_status bin_sort_views(int nv, int32_t P, const int32_t *widths, const int32_t *heights,
                         const float *means2d, const int32_t *radii, const float *depths,
                         const float *conics, const float *log_opacities, bool precise,
                         uint32_t capacity, void *workspace, size_t workspace_bytes,
                         uint32_t *sorted_ids, uint32_t *tile_ranges, uint32_t *d_num_splats,
                         uint32_t *d_view_splats, void *stream) {
    ViewTable vtab;
    uint32_t ntiles_u;
    int tbits;
    if (P < 0 || !make_views(nv, (uint32_t)P, widths, heights, vtab, ntiles_u, tbits))
        return GS_ERR_INVALID_ARG;
    if ((uint64_t)nv * (uint64_t)P >= 0x80000000ull) return GS_ERR_INVALID_ARG;
    if (!tile_ranges || !d_num_splats || !workspace || !gs::aligned(workspace, 256) ||
        !gs::aligned(tile_ranges, 4) || !gs::aligned(d_num_splats, 4))
        return GS_ERR_INVALID_ARG;
    if (d_view_splats && !gs::aligned(d_view_splats, 4)) return GS_ERR_INVALID_ARG;
    if (P > 0 && (!means2d || !radii || !depths || !gs::aligned(means2d, 8) ||
                  !gs::aligned(radii, 4) || !gs::aligned(depths, 4)))
        return GS_ERR_INVALID_ARG;
    if (precise && P > 0 && (!conics || !log_opacities || !gs::aligned(conics, 4) ||
                             !gs::aligned(log_opacities, 4)))
        return GS_ERR_INVALID_ARG;
    if (capacity >= 0x80000000u) return GS_ERR_INVALID_ARG;
    if (capacity > 0 && (!sorted_ids || !gs::aligned(sorted_ids, 4))) return GS_ERR_INVALID_ARG;
    Layout L = layout((uint32_t)nv, (uint32_t)P, capacity, precise);
    if (workspace_bytes < L.total) return GS_ERR_CAPACITY;
    hipStream_t s = (hipStream_t)stream;
    char *ws = (char *)workspace;
    auto U = [&](size_t o) { return (uint32_t *)(ws + o); };
    uint64_t *part = (uint64_t *)(ws + L.part);
    PGauss *pg = (PGauss *)(ws + L.pg);
    const int ntiles = (int)ntiles_u;
    const int n = nv * P;  // instances
    ViewDims *vdims = (ViewDims *)(ws + L.vdims);
    const ViewRef vt{nv, (uint32_t)P, vtab.W[0], vtab.H[0], vtab.gx[0], vdims};
    if (nv > 1) hipLaunchKernelGGL(k_put_views, dim3(1), dim3(GS_MAX_BIN_VIEWS), 0, s, vtab, vdims);

    if (P == 0) {
        hipLaunchKernelGGL((k_depth_keys<false, false>), dim3((2 * ntiles + 255) / 256), dim3(256), 0, s,
                           0, (const float2 *)nullptr, (const int *)nullptr,
                           (const float *)nullptr, (const float *)nullptr, (const float *)nullptr,
                           vt, (uint32_t *)nullptr, (uint32_t *)nullptr, (void *)nullptr,
                           (PGauss *)nullptr, tile_ranges, 2 * ntiles);
        // a kernel rather than a memset node, so the call can be graph-captured
        hipLaunchKernelGGL(k_set_word, dim3(1), dim3(64), 0, s, d_num_splats, 0u);
        if (d_view_splats)
            hipLaunchKernelGGL(k_view_splats, dim3(1), dim3(GS_MAX_BIN_VIEWS), 0, s,
                               (const uint32_t *)nullptr, nv, d_view_splats);
        return gs::launch_status();
    }
    const float2 *m2 = (const float2 *)means2d;
    int nthr = n > 2 * ntiles ? n : 2 * ntiles;
    // 1. depth keys, rectangles, cleared ranges; depth order of each view's
    // Gaussians
    {
        auto kk = precise ? (nv > 1 ? k_depth_keys<true, true> : k_depth_keys<true, false>)
                          : (nv > 1 ? k_depth_keys<false, true> : k_depth_keys<false, false>);
        hipLaunchKernelGGL(kk, dim3((nthr + 255) / 256), dim3(256), 0, s, n, m2, radii, depths,
                           conics, log_opacities, vt, U(L.dkey0), U(L.did0), (void *)(ws + L.rects),
                           pg, tile_ranges, 2 * ntiles);
    }
    SortBufs db{{U(L.dkey0), U(L.dkey1)}, {U(L.did0), U(L.did1)}};
    // one segment of P per view; Gaussians without splats (key DROP_KEY)
    // leave in the first pass: view v's depth order holds the n_vis[v]
    // Gaussians that have splats
    uint32_t *n_vis = U(L.nvis);
    SegTable sd{};
    sd.nseg = nv;
    sd.stride = (uint32_t)P;
    sd.n_static = (uint32_t)P;
    int dcur = radix_sort<DEPTH_ITEMS>(db, sd, L.ncols_depth, 32, U(L.hist), U(L.totals), n_vis, s);
    const uint32_t *order = db.v[dcur];
    // 2. counts in depth order, scan (+ window owners, view bounds), expansion
    uint32_t sblocks = (n + SORT_TILE - 1) / SORT_TILE;
    {
        auto kc = precise ? (nv > 1 ? k_counts<true, true> : k_counts<true, false>)
                          : (nv > 1 ? k_counts<false, true> : k_counts<false, false>);
        hipLaunchKernelGGL(kc, dim3(sblocks), dim3(COUNT_THREADS), 0, s, n, order,
                           (const void *)(ws + L.rects),
                           (uint2 *)(ws + L.rects_sorted), U(L.cnt), (const uint32_t *)n_vis, part,
                           vt);
    }
    const uint32_t win = precise ? EMIT_TILE_P : EMIT_TILE;
    static_assert((EMIT_TILE & (EMIT_TILE - 1)) == 0 && (EMIT_TILE_P & (EMIT_TILE_P - 1)) == 0,
                  "windows are powers of two");
    uint32_t *bounds = U(L.bounds);
    hipLaunchKernelGGL(k_scan_down, dim3(sblocks), dim3(COUNT_THREADS), 0, s, U(L.cnt), U(L.offs),
                       (uint32_t)n, (const uint64_t *)part, sblocks, U(L.win), L.nwin,
                       ceil_log2(win), d_num_splats, bounds, nv, (uint32_t)P);
    if (d_view_splats)
        hipLaunchKernelGGL(k_view_splats, dim3(1), dim3(GS_MAX_BIN_VIEWS), 0, s,
                           (const uint32_t *)bounds, nv, d_view_splats);
    int npass = radix_passes(tbits);
    // ids are emitted into the buffer that the last tile pass does NOT write,
    // so the sorted ids land in sorted_ids.
    uint32_t *emit_ids = (npass % 2 == 0) ? sorted_ids : U(L.tid);
    uint32_t *other_ids = (npass % 2 == 0) ? U(L.tid) : sorted_ids;
    if (capacity == 0) emit_ids = other_ids = U(L.tid);  // nothing fits
    uint32_t eblocks = (capacity + win - 1) / win;
    SegTable st{};
    st.nseg = nv;
    st.bounds = bounds;
    st.total = d_num_splats;
    st.cap = capacity;
    st.kv = nv > 1 ? vdims : nullptr;
    // One view, 3-sigma rule: the expansion also counts the first tile pass's
    // digits (for precise lists, whose expansion already stages its window
    // in LDS, this measured no faster).  The per-window counts go to the
    // first pass's output key buffer (free until that pass scatters; RADIX
    // counts per window must fit).
    const bool emit_hist = nv == 1 && !precise && eblocks > 0 &&
                           (uint64_t)RADIX * eblocks <= (uint64_t)capacity;
    const int w0 = radix_width(tbits, 0);
    // expansion, then 3. stable sort of each view's splats by tile (digits
    // of the tile index within the view), with K-bit tile keys
    auto emit_and_sort = [&](auto key_tag) {
        using K = decltype(key_tag);
        SortBufsT<K> tb{{(K *)(ws + L.tkey0), (K *)(ws + L.tkey1)}, {emit_ids, other_ids}};
        if (eblocks > 0) {
            if (precise) {
                auto kp = k_emit_precise<false, K>;
                if constexpr (sizeof(K) == 4)
                    if (nv > 1) kp = k_emit_precise<true, K>;
                hipLaunchKernelGGL(kp, dim3(eblocks), dim3(EMIT_THREADS_P), 0, s, n, order,
                                   U(L.offs), (const uint2 *)(ws + L.rects_sorted),
                                   (const PGauss *)pg, U(L.win), L.nwin, vt,
                                   (const uint32_t *)n_vis, d_num_splats, capacity, tb.k[0],
                                   emit_ids);
            } else {
                bool done = false;
                if constexpr (sizeof(K) == 4) {
                    if (nv > 1) {
                        hipLaunchKernelGGL((k_emit<true, false, K>), dim3(eblocks), dim3(EMIT_THREADS),
                                           0, s, n, order, U(L.offs),
                                           (const uint2 *)(ws + L.rects_sorted), U(L.win), L.nwin,
                                           vt, (const uint32_t *)n_vis, d_num_splats, capacity,
                                           tb.k[0], emit_ids, (1u << w0) - 1u, U(L.tkey1));
                        done = true;
                    }
                }
                if (!done) {
                    auto ke = emit_hist ? k_emit1<true, K> : k_emit1<false, K>;
                    hipLaunchKernelGGL(ke, dim3(eblocks), dim3(EMIT1_THREADS), 0, s, n, order,
                                       U(L.offs), (const uint2 *)(ws + L.rects_sorted), U(L.win),
                                       L.nwin, vt, d_num_splats, capacity, tb.k[0], emit_ids,
                                       (1u << w0) - 1u, U(L.tkey1));
                }
            }
        }
        if (tile_items((uint32_t)nv, capacity) == TILE_ITEMS_BIG)
            tile_sort<TILE_ITEMS_BIG, K>(tb, st, L.ncols_tile, tbits, emit_hist, U(L.tkey1),
                                         U(L.hist), U(L.totals), tile_ranges, (uint32_t)ntiles, s);
        else
            tile_sort<TILE_ITEMS, K>(tb, st, L.ncols_tile, tbits, emit_hist, U(L.tkey1), U(L.hist),
                                     U(L.totals), tile_ranges, (uint32_t)ntiles, s);
    };
    if (nv == 1 && ntiles <= 65536)
        emit_and_sort(uint16_t{});
    else
        emit_and_sort(uint32_t{});
    // 4. the last tile pass wrote the starts of the tiles it met (tile
    // indices are unique across views); the ends follow from them
    hipLaunchKernelGGL(k_ranges_finish, dim3((ntiles + FINISH_THREADS - 1) / FINISH_THREADS),
                       dim3(FINISH_THREADS), 0, s, tile_ranges, (uint32_t)ntiles,
                       (const uint32_t *)d_num_splats, capacity);
    return gs::launch_status();
}

}  // namespace

extern "C" gs_status gs_bin_sort(int32_t P, const float *means2d, const int32_t *radii,
                                 const float *depths, int32_t width, int32_t height,
                                 uint32_t capacity, void *workspace, size_t workspace_bytes,
                                 uint32_t *sorted_ids, uint32_t *tile_ranges,
                                 uint32_t *d_num_splats, void *stream) {
    return bin_sort_views(1, P, &width, &height, means2d, radii, depths, nullptr, nullptr, false,
                          capacity, workspace, workspace_bytes, sorted_ids, tile_ranges,
                          d_num_splats, nullptr, stream);
}

extern "C" gs_status gs_bin_sort_precise(int32_t P, const float *means2d, const int32_t *radii,
                                         const float *depths, const float *conics,
                                         const float *log_opacities, int32_t width, int32_t height,
                                         uint32_t capacity, void *workspace,
                                         size_t workspace_bytes, uint32_t *sorted_ids,
                                         uint32_t *tile_ranges, uint32_t *d_num_splats,
                                         void *stream) {
    return bin_sort_views(1, P, &width, &height, means2d, radii, depths, conics, log_opacities, true,
                          capacity, workspace, workspace_bytes, sorted_ids, tile_ranges,
                          d_num_splats, nullptr, stream);
}

extern "C" gs_status gs_bin_sort_multiview(int32_t nviews, int32_t P, const int32_t *widths,
                                           const int32_t *heights, const float *means2d,
                                           const int32_t *radii, const float *depths,
                                           const float *conics, const float *log_opacities,
                                           int32_t precise, uint32_t capacity, void *workspace,
                                           size_t workspace_bytes, uint32_t *sorted_ids,
                                           uint32_t *tile_ranges, uint32_t *d_num_splats,
                                           uint32_t *d_view_splats, void *stream) {
    return bin_sort_views(nviews, P, widths, heights, means2d, radii, depths, conics, log_opacities,
                          precise != 0, capacity, workspace, workspace_bytes, sorted_ids,
                          tile_ranges, d_num_splats, d_view_splats, stream);
}

// ---------------------------------------------------------------------------
// gs_bin_sort_noalloc: gs_bin_sort with its workspace in a file-scope device
// array, for callers that cannot allocate.  Each device the library runs on
// holds its own copy of the array until the process ends.  In host code the
// array's name is only a host-side stand-in, so its device address is looked
// up once per device (with that device current) and only that address is
// passed to kernels.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[GS_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxScratchDevices];

gs_status scratch_of_current_device(void **out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return GS_ERR_HIP;
    if (dev < 0 || dev >= kMaxScratchDevices) return GS_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return GS_ERR_HIP;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return GS_OK;
}

}  // namespace

extern "C" gs_status gs_bin_sort_noalloc(int32_t P, const float *means2d, const int32_t *radii,
                                         const float *depths, int32_t width, int32_t height,
                                         uint32_t capacity, uint32_t *sorted_ids,
                                         uint32_t *tile_ranges, uint32_t *d_num_splats,
                                         void *stream) {
    const size_t need = gs_bin_sort_workspace_bytes(P, capacity, width, height);
    if (need == 0) return GS_ERR_INVALID_ARG;
    if (need > (size_t)GS_NOALLOC_SCRATCH_BYTES) return GS_ERR_CAPACITY;
    void *ws = nullptr;
    const gs_status st = scratch_of_current_device(&ws);
    if (st != GS_OK) return st;
    return bin_sort_views(1, P, &width, &height, means2d, radii, depths, nullptr, nullptr, false,
                          capacity, ws, (size_t)GS_NOALLOC_SCRATCH_BYTES, sorted_ids, tile_ranges,
                          d_num_splats, nullptr, stream);
}
