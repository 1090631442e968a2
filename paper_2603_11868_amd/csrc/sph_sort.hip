// Device-wide exclusive scan and the stable LSD radix sort of cell keys.
//
// Radix sort (Sec. 5 of the paper sorts particles by cell with a radix sort):
// 8-bit digits, least significant first, ceil(bits(C-1)/8) passes.  Each pass
// is reduce-then-scan: per-tile digit histograms, one exclusive scan of the
// digit-major histogram table, then a scatter in which every tile ranks its
// keys stably.  Ranking inside a wave: where the wave's digits do not
// decrease from lane to lane (keys nearly in cell order, as they are between
// physical reorders), equal digits form one run, and a lane's rank is its
// distance from the head of its run; otherwise 8 ballots find the lanes that
// share a digit and v_mbcnt gives the rank among them.  Across the 4 waves of
// a block and the 16 rounds of a tile, per-digit counters in LDS keep the
// order of the input.  Ties therefore keep their input order, and the result is the
// unique stable permutation: identical to a plain counting sort of the keys.
#include "sph_launch.h"

namespace sphx {

constexpr int SCAN_BS = 256;
constexpr int SCAN_IPT = 8;
constexpr int SCAN_TILE = SCAN_BS * SCAN_IPT;
constexpr int SCAN_TOP_BS = 1024;
constexpr int SCAN_TOP_IPT = 16;

constexpr int RS_BS = 256;
constexpr int RS_IPT = 16;
constexpr int RS_TILE = RS_BS * RS_IPT;
constexpr int RS_RADIX = 256;

int scan_tiles(int64_t n) { return (int)((n + SCAN_TILE - 1) / SCAN_TILE); }
int64_t scan_max_elems() { return (int64_t)SCAN_TOP_BS * SCAN_TOP_IPT * SCAN_TILE; }
int radix_tiles(int64_t n) { return (int)((n + RS_TILE - 1) / RS_TILE); }

// The SCAN_IPT consecutive ints of thread t of the block: two 16-byte loads
// where the array is 16-byte aligned and the run lies inside it, else one by
// one (zeros past the end).
template <bool VEC>
__device__ __forceinline__ void scan_load(const int *__restrict__ in, int64_t base, int n, int (&v)[SCAN_IPT])
{
    static_assert(SCAN_IPT == 8, "two int4 per thread");
    if (VEC && base + SCAN_IPT <= n) {
        const int4 a = *reinterpret_cast<const int4 *>(in + base);
        const int4 b = *reinterpret_cast<const int4 *>(in + base + 4);
        v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
        v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
    } else {
#pragma unroll
        for (int j = 0; j < SCAN_IPT; ++j) v[j] = base + j < n ? in[base + j] : 0;
    }
}

template <bool VEC>
__global__ __launch_bounds__(SCAN_BS) void k_scan_reduce(const int *__restrict__ in, int n,
                                                         int *__restrict__ part, const int *__restrict__ gate)
{
    if (gate && *gate == 0) return;
    __shared__ int lds[SCAN_BS / 64 + 1];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_IPT;
    int v[SCAN_IPT];
    scan_load<VEC>(in, base, n, v);
    int s = 0;
#pragma unroll
    for (int j = 0; j < SCAN_IPT; ++j) s += v[j];
    int tot;
    block_exclusive_scan(s, lds, &tot);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

__global__ __launch_bounds__(SCAN_TOP_BS) void k_scan_top(int *__restrict__ part, int ntiles,
                                                           const int *__restrict__ gate)
{
    if (gate && *gate == 0) return;
    __shared__ int lds[SCAN_TOP_BS / 64 + 1];
    const int base = threadIdx.x * SCAN_TOP_IPT;
    int v[SCAN_TOP_IPT];
    int s = 0;
#pragma unroll
    for (int j = 0; j < SCAN_TOP_IPT; ++j) {
        int idx = base + j;
        v[j] = (idx < ntiles) ? part[idx] : 0;
        s += v[j];
    }
    int tot;
    int off = block_exclusive_scan(s, lds, &tot);
#pragma unroll
    for (int j = 0; j < SCAN_TOP_IPT; ++j) {
        int idx = base + j;
        if (idx < ntiles) part[idx] = off;
        off += v[j];
    }
}

template <bool VEC>
__global__ __launch_bounds__(SCAN_BS) void k_scan_apply(int *__restrict__ in, int *__restrict__ out,
                                                        int n, const int *__restrict__ part,
                                                        int zero_in, const int *__restrict__ gate)
{
    if (gate && *gate == 0) return;
    __shared__ int lds[SCAN_BS / 64 + 1];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_IPT;
    int v[SCAN_IPT];
    scan_load<VEC>(in, base, n, v);
    int s = 0;
#pragma unroll
    for (int j = 0; j < SCAN_IPT; ++j) s += v[j];
    int tot;
    int off = block_exclusive_scan(s, lds, &tot) + part[blockIdx.x];
    int o[SCAN_IPT];
#pragma unroll
    for (int j = 0; j < SCAN_IPT; ++j) {
        o[j] = off;
        off += v[j];
    }
    if (VEC && base + SCAN_IPT <= n) {
        *reinterpret_cast<int4 *>(out + base) = make_int4(o[0], o[1], o[2], o[3]);
        *reinterpret_cast<int4 *>(out + base + 4) = make_int4(o[4], o[5], o[6], o[7]);
        if (zero_in) {
            *reinterpret_cast<int4 *>(in + base) = make_int4(0, 0, 0, 0);
            *reinterpret_cast<int4 *>(in + base + 4) = make_int4(0, 0, 0, 0);
        }
    } else {
#pragma unroll
        for (int j = 0; j < SCAN_IPT; ++j) {
            if (base + j < n) {
                out[base + j] = o[j];
                if (zero_in) in[base + j] = 0;
            }
        }
    }
}

// Exclusive scan of n ints (out may alias in).  part: scan_tiles(n) ints.
hipError_t launch_exclusive_scan(int *in, int *out, int64_t n, int *part, int zero_in,
                                 hipStream_t s, const int *gate)
{
    if (n <= 0) return hipSuccess;
    if (n > scan_max_elems()) return hipErrorInvalidValue;
    int nt = scan_tiles(n);
    const bool vec = ((reinterpret_cast<uintptr_t>(in) | reinterpret_cast<uintptr_t>(out)) & 15u) == 0;
    if (vec) k_scan_reduce<true><<<nt, SCAN_BS, 0, s>>>(in, (int)n, part, gate);
    else k_scan_reduce<false><<<nt, SCAN_BS, 0, s>>>(in, (int)n, part, gate);
    k_scan_top<<<1, SCAN_TOP_BS, 0, s>>>(part, nt, gate);
    if (vec) k_scan_apply<true><<<nt, SCAN_BS, 0, s>>>(in, out, (int)n, part, zero_in, gate);
    else k_scan_apply<false><<<nt, SCAN_BS, 0, s>>>(in, out, (int)n, part, zero_in, gate);
    return hipGetLastError();
}

// Lanes of this wave whose 8-bit digit equals this lane's (valid lanes only).
__device__ __forceinline__ uint64_t match_digit(unsigned d, bool valid)
{
    uint64_t m = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        const bool bit = (d >> b) & 1u;
        const uint64_t bb = __ballot(bit);
        m &= bit ? bb : ~bb;
    }
    return m;
}

// Rank of this lane among the valid lanes of the wave with its digit d (those
// below it), and their number (valid lanes form a prefix of the wave).
struct DigitRank { int rk, cnt; };
__device__ __forceinline__ DigitRank digit_rank(unsigned d, bool valid)
{
    const int lane = lane_id();
    const unsigned dp = (unsigned)__builtin_amdgcn_ds_bpermute((lane > 0 ? lane - 1 : 0) << 2, (int)d);
    const int nvalid = __popcll(__ballot(valid));        // taken by every lane, before any branch
    DigitRank o;
    if (__ballot(valid && lane > 0 && d < dp) == 0) {
        // non-decreasing digits: runs of equal digits, one per digit
        const uint64_t heads = __ballot(valid && (lane == 0 || d != dp));
        const uint64_t upto = (2ull << lane) - 1ull;      // lanes 0..lane
        const uint64_t below = heads & upto, above = heads & ~upto;
        const int hl = 63 - __clzll(below | 1ull);
        const int nh = above ? __ffsll((long long)above) - 1 : nvalid;
        o.rk = lane - hl;
        o.cnt = nh - hl;
    } else {
        const uint64_t m = match_digit(d, valid);
        o.rk = mbcnt(m);
        o.cnt = __popcll(m);
    }
    return o;
}

// Tile of block b: blocks go to the 8 XCDs round robin, and each XCD takes a
// contiguous range of tiles, so that the runs neighbouring tiles write for a
// digit (which share memory sectors at their ends) meet in one L2.
__device__ __forceinline__ int xcd_tile(int b, int nt)
{
    const int per = nt >> 3, rem = nt & 7, x = b & 7;
    return x * per + min(x, rem) + (b >> 3);
}

__global__ __launch_bounds__(RS_BS) void k_radix_hist(const int *__restrict__ keys, int n,
                                                      int shift, int *__restrict__ hist,
                                                      int ntiles, const int *__restrict__ gate)
{
    if (gate && *gate == 0) return;
    __shared__ int h[RS_RADIX];
    const int tid = threadIdx.x;
    h[tid] = 0;
    __syncthreads();
    const int tile = xcd_tile(blockIdx.x, ntiles);
    const int64_t tbase = (int64_t)tile * RS_TILE;
    // the tile's digits: every load issued before the first is used (a
    // place past the end reads the last key and is not counted)
    unsigned dk[RS_IPT];
#pragma unroll
    for (int r = 0; r < RS_IPT; ++r)
        dk[r] = ((unsigned)keys[min(tbase + r * RS_BS + tid, (int64_t)n - 1)] >> shift) & 255u;
#pragma unroll
    for (int r = 0; r < RS_IPT; ++r) {
        const bool valid = tbase + r * RS_BS + tid < n;
        const unsigned d = valid ? dk[r] : 0u;
        const DigitRank g = digit_rank(d, valid);
        if (valid && g.rk == 0) atomicAdd(&h[d], g.cnt);
    }
    __syncthreads();
    hist[(int64_t)tid * ntiles + tile] = h[tid];
}

__global__ __launch_bounds__(RS_BS) void k_radix_scatter(const int *__restrict__ kin,
                                                         const int *__restrict__ vin, int n,
                                                         int shift,
                                                         const int *__restrict__ hist, int ntiles,
                                                         int *__restrict__ kout,
                                                         int *__restrict__ vout,
                                                         const int *__restrict__ gate)
{
    if (gate && *gate == 0) return;
    // Per-digit offsets (two copies: round r reads copy r & 1 and writes the
    // other) and per-wave digit counts (three copies: round r writes copy
    // r % 3 and clears the copy of round r - 1, whose reads all came before
    // this round's barrier and whose next writes come after the next one), so
    // that one barrier per round orders everything.
    __shared__ int base[2][RS_RADIX];
    __shared__ int wc[3][RS_BS / 64][RS_RADIX];
    const int tid = threadIdx.x;
    const int w = tid >> 6;
    const int tile = xcd_tile(blockIdx.x, ntiles);
    base[0][tid] = hist[(int64_t)tid * ntiles + tile];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int q = 0; q < RS_BS / 64; ++q) wc[c][q][tid] = 0;
    const int64_t tbase = (int64_t)tile * RS_TILE;
    // the tile's keys and values, loaded before the first round (places past
    // the end read the last element and are not written)
    int kk[RS_IPT], vv[RS_IPT];
#pragma unroll
    for (int r = 0; r < RS_IPT; ++r) {
        const int64_t idx = tbase + r * RS_BS + tid;
        const int64_t ic = min(idx, (int64_t)n - 1);
        kk[r] = kin[ic];
        vv[r] = vin ? vin[ic] : (int)idx;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < RS_IPT; ++r) {
        const int cb = r & 1, cw = r % 3, cprev = (r + 2) % 3;
        const int64_t idx = tbase + r * RS_BS + tid;
        const bool valid = idx < n;
        const int key = valid ? kk[r] : 0;
        const unsigned d = ((unsigned)key >> shift) & 255u;
        const DigitRank g = digit_rank(d, valid);
        if (valid && g.rk == 0) wc[cw][w][d] = g.cnt;
        __syncthreads();
        int pos = 0;
        if (valid) {
            pos = base[cb][d] + g.rk;
#pragma unroll
            for (int q = 0; q < RS_BS / 64; ++q) pos += q < w ? wc[cw][q][d] : 0;
        }
        int add = 0;
#pragma unroll
        for (int q = 0; q < RS_BS / 64; ++q) {
            add += wc[cw][q][tid];
            wc[cprev][q][tid] = 0;
        }
        base[cb ^ 1][tid] = base[cb][tid] + add;
        if (valid) {
            kout[pos] = key;
            vout[pos] = vv[r];
        }
    }
}

int radix_passes(int64_t ncells)
{
    int bits = 1;
    while (bits < 31 && ((int64_t)1 << bits) < ncells) ++bits;
    return (bits + 7) / 8;
}

// Stable sort of indices 0..n-1 by keys[] (values < ncells).  Writes the
// sorted keys to skey and the permutation to perm.  Scratch: k0, v0, k1, v1
// (n ints each), hist (RS_RADIX * radix_tiles(n)), part (scan tiles).
hipError_t launch_radix_sort(const int *keys, int64_t n, int64_t ncells, int *skey, int *perm,
                             int *k0, int *v0, int *k1, int *v1, int *hist, int *part,
                             hipStream_t s, const int *gate)
{
    if (n <= 0) return hipSuccess;
    const int nt = radix_tiles(n);
    const int passes = radix_passes(ncells);
    const int *kin = keys;
    const int *vin = nullptr;
    for (int p = 0; p < passes; ++p) {
        const int shift = 8 * p;
        int *ko, *vo;
        if (p == passes - 1) { ko = skey; vo = perm; }
        else if (p % 2 == 0) { ko = k0; vo = v0; }
        else { ko = k1; vo = v1; }
        k_radix_hist<<<nt, RS_BS, 0, s>>>(kin, (int)n, shift, hist, nt, gate);
        hipError_t e = launch_exclusive_scan(hist, hist, (int64_t)RS_RADIX * nt, part, 0, s, gate);
        if (e != hipSuccess) return e;
        k_radix_scatter<<<nt, RS_BS, 0, s>>>(kin, vin, (int)n, shift, hist, nt, ko, vo, gate);
        kin = ko;
        vin = vo;
    }
    return hipGetLastError();
}

}  // namespace sphx
