// Device-wide exclusive scan and a stable LSD radix sort (key/value), both
// written for wave64: the per-block scans use wave shuffles plus one LDS
// exchange between the four waves of a block, and the sort ranks keys inside
// a wave with eight ballots (one per digit bit), so each pass is stable and
// the whole sort is deterministic.
#include "crk_internal.h"

namespace crk {
namespace {

constexpr int kScanItems = 8;                       // per thread
constexpr int kScanTile = kBlock * kScanItems;      // 2048 per block

// inclusive scan of one value per thread across a 256-thread block
template <typename T>
__device__ T block_inclusive_scan(T v, T *lds /* [4] */) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        T u = __shfl_up(v, o, 64);
        if (lane >= o) v += u;
    }
    if (lane == 63) lds[w] = v;
    __syncthreads();
    T add = 0;
    for (int k = 0; k < w; k++) add += lds[k];
    __syncthreads();
    return v + add;
}

__global__ __launch_bounds__(kBlock) void k_scan_sums(const int64_t *in, int64_t n, int64_t *bsum) {
    __shared__ int64_t lds[4];
    int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int64_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; k++)
        if (base + k < n) s += in[base + k];
    s = block_inclusive_scan(s, lds);
    if (threadIdx.x == kBlock - 1) bsum[blockIdx.x] = s;
}

__global__ __launch_bounds__(kBlock) void k_scan_apply(const int64_t *in, int64_t *out, int64_t n,
                                                       const int64_t *boff) {
    __shared__ int64_t lds[4];
    int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int64_t v[kScanItems];
    int64_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; k++) {
        v[k] = (base + k < n) ? in[base + k] : 0;
        s += v[k];
    }
    int64_t incl = block_inclusive_scan(s, lds);
    int64_t run = incl - s + (boff ? boff[blockIdx.x] : 0);
#pragma unroll
    for (int k = 0; k < kScanItems; k++) {
        if (base + k < n) out[base + k] = run;
        run += v[k];
    }
}

// The same two kernels for a pair of int32 count arrays (blockIdx.y picks
// the array): each array's first nin values, then zeros up to nout, scanned
// into int64 offsets, so the offsets of n rows come out with the total as
// their (n + 1)-th entry without a widening copy first.
// largest value of one per thread across a 256-thread block (thread 0 holds it)
__device__ int64_t block_max(int64_t v, int64_t *lds /* [4] */) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const int64_t u = __shfl_xor(v, o, 64);
        v = u > v ? u : v;
    }
    __syncthreads();
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0)
        for (int k = 1; k < kBlock / 64; k++) v = lds[k] > v ? lds[k] : v;
    return v;
}

// a thread's kScanItems (8) consecutive int32 inputs, zeros past nin; VEC:
// two 16-byte loads where all eight are in range (the array 16-byte aligned)
template <bool VEC>
__device__ __forceinline__ void load8(const int32_t *in, int64_t base, int64_t nin, int64_t v[8]) {
    if (VEC && base + 8 <= nin) {
        const int4 a = *(const int4 *)(in + base), b = *(const int4 *)(in + base + 4);
        v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
        v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
    } else {
#pragma unroll
        for (int k = 0; k < 8; k++) v[k] = base + k < nin ? (int64_t)in[base + k] : 0;
    }
}

// (with bm: also each block's largest value of the first array)
template <bool VEC>
__global__ __launch_bounds__(kBlock) void k_scan_sums2(const int32_t *in0, const int32_t *in1, int64_t nin,
                                                       int64_t *bs0, int64_t *bs1, int64_t *bm) {
    static_assert(kScanItems == 8, "eight items per thread");
    __shared__ int64_t lds[4];
    const int32_t *in = blockIdx.y ? in1 : in0;
    int64_t *bsum = blockIdx.y ? bs1 : bs0;
    int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int64_t v[8];
    load8<VEC>(in, base, nin, v);
    int64_t s = 0, mx = 0;
#pragma unroll
    for (int k = 0; k < 8; k++) {
        s += v[k];
        mx = v[k] > mx ? v[k] : mx;
    }
    s = block_inclusive_scan(s, lds);
    if (threadIdx.x == kBlock - 1) bsum[blockIdx.x] = s;
    if (bm && blockIdx.y == 0) {
        mx = block_max(mx, lds);
        if (threadIdx.x == 0) bm[blockIdx.x] = mx;
    }
}

// the largest of m block maxima (one block)
__global__ __launch_bounds__(kBlock) void k_max_i64(const int64_t *bm, int64_t m, int64_t *out) {
    __shared__ int64_t lds[4];
    int64_t mx = 0;
    for (int64_t k = threadIdx.x; k < m; k += kBlock) mx = bm[k] > mx ? bm[k] : mx;
    mx = block_max(mx, lds);
    if (threadIdx.x == 0) *out = mx;
}

// (with o32: the first nin offsets of the second array also as int32)
template <bool VEC>
__global__ __launch_bounds__(kBlock) void k_scan_apply2(const int32_t *in0, const int32_t *in1, int64_t nin,
                                                        int64_t nout, int64_t *out0, int64_t *out1,
                                                        const int64_t *bo0, const int64_t *bo1,
                                                        int32_t *o32) {
    __shared__ int64_t lds[4];
    const int32_t *in = blockIdx.y ? in1 : in0;
    int64_t *out = blockIdx.y ? out1 : out0;
    const int64_t *boff = blockIdx.y ? bo1 : bo0;
    int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int64_t v[8];
    load8<VEC>(in, base, nin, v);
    int64_t s = 0;
#pragma unroll
    for (int k = 0; k < 8; k++) s += v[k];
    int64_t incl = block_inclusive_scan(s, lds);
    int64_t run = incl - s + boff[blockIdx.x];
    int64_t o[8];
#pragma unroll
    for (int k = 0; k < 8; k++) {
        o[k] = run;
        run += v[k];
    }
    if (VEC && base + 8 <= nout) {
        // four 16-byte stores (the output 16-byte aligned, base a multiple of 8)
#pragma unroll
        for (int k = 0; k < 8; k += 2) *(longlong2 *)(out + base + k) = make_longlong2(o[k], o[k + 1]);
    } else {
#pragma unroll
        for (int k = 0; k < 8; k++)
            if (base + k < nout) out[base + k] = o[k];
    }
    if (o32 && blockIdx.y == 1) {
        if (VEC && base + 8 <= nin) {
            *(int4 *)(o32 + base) = make_int4((int32_t)o[0], (int32_t)o[1], (int32_t)o[2], (int32_t)o[3]);
            *(int4 *)(o32 + base + 4) = make_int4((int32_t)o[4], (int32_t)o[5], (int32_t)o[6], (int32_t)o[7]);
        } else {
#pragma unroll
            for (int k = 0; k < 8; k++)
                if (base + k < nin) o32[base + k] = (int32_t)o[k];
        }
    }
}

// block sums of both arrays scanned in place in one single-block launch
__global__ __launch_bounds__(kBlock) void k_scan_bsum2(int64_t *bs0, int64_t *bs1, int64_t m) {
    __shared__ int64_t lds[4];
    int64_t *b = blockIdx.y ? bs1 : bs0;
    int64_t v[kScanItems];
    int64_t s = 0;
    const int64_t base = (int64_t)threadIdx.x * kScanItems;
#pragma unroll
    for (int k = 0; k < kScanItems; k++) {
        v[k] = (base + k < m) ? b[base + k] : 0;
        s += v[k];
    }
    int64_t run = block_inclusive_scan(s, lds) - s;
#pragma unroll
    for (int k = 0; k < kScanItems; k++) {
        if (base + k < m) b[base + k] = run;
        run += v[k];
    }
}

// ---------------------------------------------------------------- radix sort
constexpr int kRadixBits = 8;
constexpr int kBuckets = 1 << kRadixBits;
constexpr int kSortItems = 8;                       // rounds of 256 per block
constexpr int kSortTile = kBlock * kSortItems;

__global__ __launch_bounds__(kBlock) void k_radix_hist(const uint32_t *keys, int64_t n, int shift,
                                                       int64_t nblk, int64_t *hist) {
    __shared__ int cnt[kBuckets];
    cnt[threadIdx.x] = 0;
    __syncthreads();
    int64_t base = (int64_t)blockIdx.x * kSortTile;
    for (int r = 0; r < kSortItems; r++) {
        int64_t i = base + (int64_t)r * kBlock + threadIdx.x;
        if (i < n) atomicAdd(&cnt[(keys[i] >> shift) & (kBuckets - 1)], 1);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nblk + blockIdx.x] = cnt[threadIdx.x];
}

__global__ __launch_bounds__(kBlock) void k_radix_scatter(const uint32_t *kin, const int32_t *vin,
                                                          uint32_t *kout, int32_t *vout, int64_t n,
                                                          int shift, int64_t nblk,
                                                          const int64_t *offs) {
    __shared__ int64_t base[kBuckets];
    __shared__ int wcnt[4][kBuckets];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    base[tid] = offs[(int64_t)tid * nblk + blockIdx.x];
    for (int k = 0; k < 4; k++) wcnt[k][tid] = 0;
    __syncthreads();
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    int64_t tile = (int64_t)blockIdx.x * kSortTile;
    for (int r = 0; r < kSortItems; r++) {
        int64_t i = tile + (int64_t)r * kBlock + tid;
        bool valid = i < n;
        uint32_t key = valid ? kin[i] : 0u;
        int d = (key >> shift) & (kBuckets - 1);
        // lanes of this wave holding the same digit
        uint64_t mask = __ballot(valid);
#pragma unroll
        for (int b = 0; b < kRadixBits; b++) {
            uint64_t bb = __ballot((d >> b) & 1);
            mask &= ((d >> b) & 1) ? bb : ~bb;
        }
        int rank = __popcll(mask & lt);
        if (valid && rank == 0) wcnt[w][d] = __popcll(mask);
        __syncthreads();
        int64_t pos = 0;
        if (valid) {
            int pre = 0;
            for (int k = 0; k < w; k++) pre += wcnt[k][d];
            pos = base[d] + pre + rank;
        }
        __syncthreads();
        base[tid] += wcnt[0][tid] + wcnt[1][tid] + wcnt[2][tid] + wcnt[3][tid];
        wcnt[0][tid] = wcnt[1][tid] = wcnt[2][tid] = wcnt[3][tid] = 0;
        __syncthreads();
        if (valid) {
            kout[pos] = key;
            vout[pos] = vin[i];
        }
    }
}

}  // namespace

// exclusive scan with its block sums at tmp (room for the sum over levels
// of ceil(n / 2048^k), k >= 1, plus 16)
static crk_status scan_with(crk_ctx *c, const int64_t *in, int64_t *out, int64_t n, int64_t *bsum) {
    if (n <= 0) return CRK_OK;
    int64_t nblk = (n + kScanTile - 1) / kScanTile;
    if (nblk == 1) {
        k_scan_apply<<<1, kBlock, 0, c->stream>>>(in, out, n, nullptr);
        CRK_HIP(c, hipGetLastError());
        return CRK_OK;
    }
    k_scan_sums<<<(unsigned)nblk, kBlock, 0, c->stream>>>(in, n, bsum);
    CRK_HIP(c, hipGetLastError());
    // scan the block sums in place (recursion on a disjoint region is not
    // needed: in == out is allowed by k_scan_apply's read-then-write tiles)
    {
        int64_t m = nblk;
        int64_t mblk = (m + kScanTile - 1) / kScanTile;
        if (mblk == 1) {
            k_scan_apply<<<1, kBlock, 0, c->stream>>>(bsum, bsum, m, nullptr);
            CRK_HIP(c, hipGetLastError());
        } else {
            // two-level: nblk <= 2048^2 covers n up to 8.6e9 elements
            int64_t *bsum2 = bsum + nblk;
            k_scan_sums<<<(unsigned)mblk, kBlock, 0, c->stream>>>(bsum, m, bsum2);
            CRK_HIP(c, hipGetLastError());
            if (mblk > kScanTile) return set_err(c, CRK_ERR_INVALID_ARG, "scan too large");
            k_scan_apply<<<1, kBlock, 0, c->stream>>>(bsum2, bsum2, mblk, nullptr);
            k_scan_apply<<<(unsigned)mblk, kBlock, 0, c->stream>>>(bsum, bsum, m, bsum2);
            CRK_HIP(c, hipGetLastError());
        }
    }
    k_scan_apply<<<(unsigned)nblk, kBlock, 0, c->stream>>>(in, out, n, bsum);
    CRK_HIP(c, hipGetLastError());
    return CRK_OK;
}

static size_t scan_need(int64_t n) {
    size_t need = 0;
    for (int64_t m = (n + kScanTile - 1) / kScanTile; m > 1; m = (m + kScanTile - 1) / kScanTile)
        need += (size_t)m;
    return need;
}

crk_status scan_exclusive_i64(crk_ctx *c, const int64_t *in, int64_t *out, int64_t n) {
    if (n <= 0) return CRK_OK;
    // block sums live in a scratch buffer; the recursion uses the tail of it
    CRK_TRY(ensure(c, c->scanTmp, (scan_need(n) + 16) * sizeof(int64_t)));
    return scan_with(c, in, out, n, (int64_t *)c->scanTmp.p);
}

crk_status scan_counts2(crk_ctx *c, const int32_t *a, const int32_t *b, int64_t n, int64_t *oa,
                        int64_t *ob, int64_t *amax, int32_t *ob32) {
    if (n < 0) return set_err(c, CRK_ERR_INVALID_ARG, "negative count");
    if ((b == nullptr) != (ob == nullptr) || (ob32 && !b))
        return set_err(c, CRK_ERR_INVALID_ARG, "scan_counts2: b, ob and ob32 do not match");
    const unsigned ny = b ? 2u : 1u;
    const int64_t nout = n + 1, nblk = (nout + kScanTile - 1) / kScanTile;
    const size_t need = scan_need(nblk);
    CRK_TRY(ensure(c, c->scanTmp, (3 * (size_t)nblk + need + 16) * sizeof(int64_t)));
    int64_t *bs0 = (int64_t *)c->scanTmp.p, *bs1 = bs0 + nblk, *bm = bs1 + nblk, *tail = bm + nblk;
    auto al16 = [](const void *q) { return ((uintptr_t)q & 15u) == 0; };
    const bool vec = al16(a) && al16(oa) && (!b || (al16(b) && al16(ob))) && (!ob32 || al16(ob32));
    if (vec)
        k_scan_sums2<true><<<dim3((unsigned)nblk, ny), kBlock, 0, c->stream>>>(a, b, n, bs0, bs1, amax ? bm : nullptr);
    else
        k_scan_sums2<false><<<dim3((unsigned)nblk, ny), kBlock, 0, c->stream>>>(a, b, n, bs0, bs1, amax ? bm : nullptr);
    CRK_HIP(c, hipGetLastError());
    if (amax) k_max_i64<<<1, kBlock, 0, c->stream>>>(bm, nblk, amax);
    if (nblk <= kScanTile) {
        k_scan_bsum2<<<dim3(1, ny), kBlock, 0, c->stream>>>(bs0, bs1, nblk);
        CRK_HIP(c, hipGetLastError());
    } else {
        CRK_TRY(scan_with(c, bs0, bs0, nblk, tail));
        if (b) CRK_TRY(scan_with(c, bs1, bs1, nblk, tail));
    }
    if (vec)
        k_scan_apply2<true><<<dim3((unsigned)nblk, ny), kBlock, 0, c->stream>>>(a, b, n, nout, oa, ob, bs0, bs1, ob32);
    else
        k_scan_apply2<false><<<dim3((unsigned)nblk, ny), kBlock, 0, c->stream>>>(a, b, n, nout, oa, ob, bs0, bs1, ob32);
    CRK_HIP(c, hipGetLastError());
    return CRK_OK;
}

crk_status radix_sort_pairs(crk_ctx *c, uint32_t *keys, int32_t *vals, int64_t n, int bits) {
    if (n <= 1 || bits <= 0) return CRK_OK;
    int64_t nblk = (n + kSortTile - 1) / kSortTile;
    CRK_TRY(ensure(c, c->keyB, (size_t)n * sizeof(uint32_t)));
    CRK_TRY(ensure(c, c->valB, (size_t)n * sizeof(int32_t)));
    CRK_TRY(ensure(c, c->hist, (size_t)nblk * kBuckets * sizeof(int64_t)));
    uint32_t *ka = keys, *kb = (uint32_t *)c->keyB.p;
    int32_t *va = vals, *vb = (int32_t *)c->valB.p;
    int64_t *hist = (int64_t *)c->hist.p;
    int passes = (bits + kRadixBits - 1) / kRadixBits;
    for (int p = 0; p < passes; p++) {
        int shift = p * kRadixBits;
        k_radix_hist<<<(unsigned)nblk, kBlock, 0, c->stream>>>(ka, n, shift, nblk, hist);
        CRK_HIP(c, hipGetLastError());
        CRK_TRY(scan_exclusive_i64(c, hist, hist, nblk * kBuckets));
        k_radix_scatter<<<(unsigned)nblk, kBlock, 0, c->stream>>>(ka, va, kb, vb, n, shift, nblk, hist);
        CRK_HIP(c, hipGetLastError());
        uint32_t *tk = ka; ka = kb; kb = tk;
        int32_t *tv = va; va = vb; vb = tv;
    }
    if (ka != keys) {
        CRK_HIP(c, hipMemcpyAsync(keys, ka, (size_t)n * sizeof(uint32_t), hipMemcpyDeviceToDevice, c->stream));
        CRK_HIP(c, hipMemcpyAsync(vals, va, (size_t)n * sizeof(int32_t), hipMemcpyDeviceToDevice, c->stream));
    }
    return CRK_OK;
}

}  // namespace crk
