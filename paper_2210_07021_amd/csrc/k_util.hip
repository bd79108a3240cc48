// Generic device building blocks: fills, exclusive scan, stable LSD radix
// sort, deterministic reduction, and the caching device allocator.
#include "common.hpp"

#include <map>
#include <memory>
#include <mutex>
#include <unordered_map>

namespace sfmm {

// ------------------------------------------------------------------ pool
// A freed block is not handed out again until the work that may still use
// it has finished.  Each API call is one epoch on its stream (PoolStream):
// blocks freed during the call belong to it, and when the call ends one
// event is recorded on the stream for the whole epoch (the last use of each
// of its blocks was queued before that).  A cached block is reused by an
// allocation on the stream of its epoch at once (stream order covers it),
// by one on any other stream only once its epoch has ended and the event
// has completed.  Blocks are kept per device.  While a stream is being
// captured into a graph its frees are retired instead (graph replays may
// still use them); they are released with the pool.
namespace {
struct Epoch {
    hipStream_t s = nullptr;
    hipEvent_t ev = nullptr;
    bool ended = false;   // the event is recorded
    bool waited = false;  // ... and has completed
    Epoch() = default;
    Epoch(const Epoch&) = delete;
    Epoch& operator=(const Epoch&) = delete;
    ~Epoch() {
        if (ev) (void)hipEventDestroy(ev);
    }
};
struct FreeBlock {
    void* p;
    int dev;
    std::shared_ptr<Epoch> ep;  // null: reusable at once
};
std::mutex g_pool_mu;
// never destroyed: the blocks' events must not be released after the HIP
// runtime has shut down at process exit
std::multimap<size_t, FreeBlock>& g_free = *new std::multimap<size_t, FreeBlock>;  // size -> block
std::unordered_map<void*, std::pair<size_t, int>> g_size;  // live and free blocks: size, device
std::vector<void*> g_retired;
struct ThreadScope {
    std::shared_ptr<Epoch> ep;
    bool capturing = false, idle = false, used = false;
};
thread_local ThreadScope t_scope;
}  // namespace

PoolStream::PoolStream(hipStream_t s, bool capturing, bool idle) {
    auto* prev = new ThreadScope(t_scope);
    saved = prev;
    t_scope = ThreadScope{};
    t_scope.ep = std::make_shared<Epoch>();
    t_scope.ep->s = s;
    t_scope.capturing = capturing;
    t_scope.idle = idle;
}

PoolStream::~PoolStream() {
    // end the epoch: one event covers every block freed in it
    if (t_scope.used && !t_scope.idle && !t_scope.capturing) {
        std::lock_guard<std::mutex> lk(g_pool_mu);
        Epoch& e = *t_scope.ep;
        if (hipEventCreateWithFlags(&e.ev, hipEventDisableTiming) == hipSuccess &&
            hipEventRecord(e.ev, e.s) == hipSuccess) {
            e.ended = true;
        } else {
            (void)hipGetLastError();  // never ended: its blocks serve only their own stream
        }
    }
    auto* prev = static_cast<ThreadScope*>(saved);
    t_scope = *prev;
    delete prev;
}

static size_t size_class(size_t b) {
    if (b < 512) return 512;
    // round up to 1/8 of the next power of two
    size_t p = 1;
    while (p < b) p <<= 1;
    const size_t step = p >> 3;
    return (b + step - 1) / step * step;
}

void* pool_alloc(size_t bytes) {
    const size_t sz = size_class(bytes);
    int dev = 0;
    SFMM_HIP(hipGetDevice(&dev));
    hipStream_t cur = t_scope.ep ? t_scope.ep->s : nullptr;
    {
        std::lock_guard<std::mutex> lk(g_pool_mu);
        for (auto it = g_free.lower_bound(sz); it != g_free.end() && it->first <= 2 * sz; ++it) {
            const FreeBlock& b = it->second;
            PoolBlockState st{b.dev, b.ep ? b.ep->s : nullptr, b.ep != nullptr && !b.ep->waited, false};
            if (st.has_event && st.s != cur && b.dev == dev && b.ep->ended) {
                const hipError_t q = hipEventQuery(b.ep->ev);
                if (q != hipSuccess && q != hipErrorNotReady) (void)hipGetLastError();
                if (q == hipSuccess) b.ep->waited = true;
                st.event_done = q == hipSuccess;
            }
            if (!pool_reusable(st, cur, dev)) continue;
            void* p = b.p;
            g_free.erase(it);
            return p;
        }
    }
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, sz);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        pool_release_all();
        e = hipMalloc(&p, sz);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            throw Error(ST_OOM, "device allocation of " + std::to_string(sz) + " bytes failed");
        }
    }
    std::lock_guard<std::mutex> lk(g_pool_mu);
    g_size[p] = {sz, dev};
    return p;
}

void pool_free(void* p) {
    if (!p) return;
    std::lock_guard<std::mutex> lk(g_pool_mu);
    auto it = g_size.find(p);
    if (it == g_size.end()) return;
    if (t_scope.capturing) {
        g_retired.push_back(p);
        return;
    }
    FreeBlock b{p, it->second.second, nullptr};
    if (!t_scope.idle) {
        if (!t_scope.ep) t_scope.ep = std::make_shared<Epoch>();  // outside any API call: the null stream
        b.ep = t_scope.ep;
        t_scope.used = true;
    }
    g_free.emplace(it->second.first, b);
}

void pool_release_all() {
    // blocks whose last users may still run are waited for first
    (void)hipDeviceSynchronize();
    std::lock_guard<std::mutex> lk(g_pool_mu);
    for (auto& kv : g_free) {
        (void)hipFree(kv.second.p);
        g_size.erase(kv.second.p);
    }
    g_free.clear();
}

// ------------------------------------------------------------------ fills
template <typename T>
__global__ void k_fill(T* p, size_t n, T v) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}

static unsigned grid_for(size_t n, unsigned block, unsigned cap = 65536) {
    size_t g = (n + block - 1) / block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}

void fill_f64(double* p, size_t n, double v, hipStream_t s) {
    if (!n) return;
    k_fill<double><<<grid_for(n, 256), 256, 0, s>>>(p, n, v);
    SFMM_LAUNCH_CHECK();
}

void fill_f32(float* p, size_t n, float v, hipStream_t s) {
    if (!n) return;
    k_fill<float><<<grid_for(n, 256), 256, 0, s>>>(p, n, v);
    SFMM_LAUNCH_CHECK();
}

void fill_i32(int* p, size_t n, int v, hipStream_t s) {
    if (!n) return;
    k_fill<int><<<grid_for(n, 256), 256, 0, s>>>(p, n, v);
    SFMM_LAUNCH_CHECK();
}

// ------------------------------------------------------------------ scan
constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanThreads * kScanItems;

// block-wide exclusive scan of one value per thread (256 threads = 4 waves):
// inclusive scan inside each wave by shuffles, then the wave totals
__device__ int block_excl_scan(int v, int* sh, int* total) {
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    int x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) sh[wv] = x;
    __syncthreads();
    int before = 0, all = 0;
#pragma unroll
    for (int w = 0; w < kScanThreads / 64; ++w) {
        const int ws = sh[w];
        before += (w < wv) ? ws : 0;
        all += ws;
    }
    *total = all;
    __syncthreads();  // sh may be reused by the caller
    return before + x - v;
}

__global__ void k_scan_tiles(const int* in, int* out, int64_t n, int* bsum) {
    __shared__ int sh[kScanThreads / 64];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int v[kScanItems];
    int s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        v[k] = (base + k < n) ? in[base + k] : 0;
        s += v[k];
    }
    int tot;
    int run = block_excl_scan(s, sh, &tot);
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        if (base + k < n) out[base + k] = run;
        run += v[k];
    }
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__global__ void k_scan_add(int* out, int64_t n, const int* boff) {
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    const int add = boff[blockIdx.x];
    for (int k = threadIdx.x; k < kScanTile; k += kScanThreads)
        if (base + k < n) out[base + k] += add;
}

// Three scans of n ints at once (blockIdx.y picks the array): the same tile
// scan / block-sum scan / add-back as scan_excl_i32, a third of the launches.
struct Scan3 {
    const int* in[3];
    int* out[3];
    int* aux[3];  // tile sums (or the totals, with a single tile)
};

__global__ void k_scan_tiles3(Scan3 a, int64_t n) {
    __shared__ int sh[kScanThreads / 64];
    const int j = blockIdx.y;
    const int* in = a.in[j];
    int* out = a.out[j];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int v[kScanItems];
    int s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        v[k] = (base + k < n) ? in[base + k] : 0;
        s += v[k];
    }
    int tot;
    int run = block_excl_scan(s, sh, &tot);
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        if (base + k < n) out[base + k] = run;
        run += v[k];
    }
    if (threadIdx.x == 0) a.aux[j][blockIdx.x] = tot;
}

__global__ void k_scan_add3(Scan3 a, int64_t n) {
    const int j = blockIdx.y;
    int* out = a.out[j];
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    const int add = a.aux[j][blockIdx.x];
    for (int k = threadIdx.x; k < kScanTile; k += kScanThreads)
        if (base + k < n) out[base + k] += add;
}

void scan3_excl_i32(const int* in0, const int* in1, const int* in2, int* out0, int* out1, int* out2, int64_t n,
                    int* total, hipStream_t s) {
    if (n <= 0) {
        fill_i32(total, 3, 0, s);
        return;
    }
    const int64_t nb = (n + kScanTile - 1) / kScanTile;
    Scan3 a{{in0, in1, in2}, {out0, out1, out2}, {total, total + 1, total + 2}};
    if (nb == 1) {
        k_scan_tiles3<<<dim3(1, 3), kScanThreads, 0, s>>>(a, n);
        SFMM_LAUNCH_CHECK();
        return;
    }
    int* bsum = (int*)pool_alloc(sizeof(int) * 3 * nb);
    int* boff = (int*)pool_alloc(sizeof(int) * 3 * nb);
    for (int j = 0; j < 3; ++j) a.aux[j] = bsum + j * nb;
    k_scan_tiles3<<<dim3((unsigned)nb, 3), kScanThreads, 0, s>>>(a, n);
    SFMM_LAUNCH_CHECK();
    scan3_excl_i32(bsum, bsum + nb, bsum + 2 * nb, boff, boff + nb, boff + 2 * nb, nb, total, s);
    for (int j = 0; j < 3; ++j) a.aux[j] = boff + j * nb;
    k_scan_add3<<<dim3((unsigned)nb, 3), kScanThreads, 0, s>>>(a, n);
    SFMM_LAUNCH_CHECK();
    // freed blocks are only reused by later stream-ordered work on this stream
    pool_free(bsum);
    pool_free(boff);
}

// Tile scans write each tile's sum to bsum; with a single tile that sum is
// the total.  Otherwise the tile sums are scanned (their total is the total)
// and added back.  In place (in == out) is allowed.
void scan_excl_i32(const int* in, int* out, int64_t n, int* total, hipStream_t s) {
    if (n <= 0) {
        fill_i32(total, 1, 0, s);
        return;
    }
    const int64_t nb = (n + kScanTile - 1) / kScanTile;
    if (nb == 1) {
        k_scan_tiles<<<1, kScanThreads, 0, s>>>(in, out, n, total);
        SFMM_LAUNCH_CHECK();
        return;
    }
    int* bsum = (int*)pool_alloc(sizeof(int) * nb);
    int* boff = (int*)pool_alloc(sizeof(int) * nb);
    k_scan_tiles<<<(unsigned)nb, kScanThreads, 0, s>>>(in, out, n, bsum);
    SFMM_LAUNCH_CHECK();
    scan_excl_i32(bsum, boff, nb, total, s);
    k_scan_add<<<(unsigned)nb, kScanThreads, 0, s>>>(out, n, boff);
    SFMM_LAUNCH_CHECK();
    // freed blocks are only reused by later stream-ordered work on this stream
    pool_free(bsum);
    pool_free(boff);
}

// ------------------------------------------------------------------ radix sort
// 8-bit digits.  Pass = histogram per tile, exclusive scan of the
// digit-major histogram, stable scatter.  Ranks inside a tile come from
// wave ballots: lanes holding the same digit are found by intersecting the
// ballots of the digit's 8 bits.
constexpr int kRsThreads = 256;
constexpr int kRsRounds = 8;
constexpr int kRsTile = kRsThreads * kRsRounds;
constexpr int kRsWaves = kRsThreads / 64;

__global__ void k_rs_hist(const uint64_t* keys, int64_t n, int shift, int rs, int* hist) {
    __shared__ int h[256];
    h[threadIdx.x] = 0;
    const int64_t base = (int64_t)blockIdx.x * kRsTile;
    int d[kRsRounds];
#pragma unroll
    for (int r = 0; r < kRsRounds; ++r) {
        const int64_t i = base + r * kRsThreads + threadIdx.x;
        d[r] = i < n ? (int)((keys[i] >> shift) & 255) : -1;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kRsRounds; ++r)
        if (d[r] >= 0) atomicAdd(&h[d[r]], 1);
    __syncthreads();
    hist[threadIdx.x * rs + blockIdx.x] = h[threadIdx.x];
}

// Exclusive scan of each digit's row of the digit-major histogram (one
// workgroup per digit, chunks of kScanTile with a running carry); dtot[d] =
// the digit's total count.  Rows are rs ints apart (rs a multiple of 4, the
// entries past nblk unused), so each thread moves its 16 entries as four
// 16-byte vectors.  The digit bases (scan of dtot) are added by the scatter.
__global__ void __launch_bounds__(kScanThreads) k_rs_rowscan(const int* __restrict__ hist, int nblk, int rs,
                                                             int* __restrict__ offs, int* __restrict__ dtot) {
    static_assert(kScanItems == 16, "four int4 per thread");
    __shared__ int sh[kScanThreads / 64];
    const int d = blockIdx.x;
    const int* in = hist + (size_t)d * rs;
    int* out = offs + (size_t)d * rs;
    int carry = 0;
    for (int c0 = 0; c0 < nblk; c0 += kScanTile) {
        const int base = c0 + threadIdx.x * kScanItems;
        int v[kScanItems];
        int sum = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            int4 x = make_int4(0, 0, 0, 0);
            if (base + 4 * q < nblk) x = *reinterpret_cast<const int4*>(in + base + 4 * q);  // within the row of rs
            v[4 * q + 0] = base + 4 * q + 0 < nblk ? x.x : 0;
            v[4 * q + 1] = base + 4 * q + 1 < nblk ? x.y : 0;
            v[4 * q + 2] = base + 4 * q + 2 < nblk ? x.z : 0;
            v[4 * q + 3] = base + 4 * q + 3 < nblk ? x.w : 0;
        }
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) sum += v[k];
        int tot;
        int run = carry + block_excl_scan(sum, sh, &tot);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            int4 o;
            o.x = run;
            run += v[4 * q + 0];
            o.y = run;
            run += v[4 * q + 1];
            o.z = run;
            run += v[4 * q + 2];
            o.w = run;
            run += v[4 * q + 3];
            if (base + 4 * q < nblk) *reinterpret_cast<int4*>(out + base + 4 * q) = o;
        }
        carry += tot;
    }
    if (threadIdx.x == 0) dtot[d] = carry;
}

// Stable scatter of one tile of kRsTile keys.  Wave w owns the tile's w-th
// quarter and walks it in rounds of 64 keys: lanes with equal digits find
// each other by ballots over the digit's bits, and a wave-private count per
// digit gives every key its rank among the equal digits before it in the
// quarter.  One pass over the counts of the four waves then places each key
// in the tile sorted by digit (LDS), and the sorted tile is written out, so
// consecutive lanes write consecutive addresses within each digit's run.
// lo_out / hi_out (the last pass of a split sort): the key's two 32-bit
// halves go to two arrays instead of the key to kout.
__global__ void __launch_bounds__(kRsThreads) k_rs_scatter(const uint64_t* kin, const uint32_t* vin, uint64_t* kout,
                                                           uint32_t* vout, int64_t n, int shift, int rs,
                                                           const int* offs, const int* dtot, uint32_t* lo_out,
                                                           uint32_t* hi_out) {
    __shared__ int wcnt[kRsWaves][256];  // per-wave digit counts, then each wave's first slot per digit
    __shared__ int goff[256];            // global position of slot 0 of each digit's run of this tile
    __shared__ int wsum[kRsWaves];
    __shared__ uint64_t sk[kRsTile];
    __shared__ uint32_t sv[kRsTile];
    const int t = threadIdx.x;
    const int wave = t >> 6, lane = t & 63;
    constexpr int kQuarter = kRsTile / kRsWaves;
#pragma unroll
    for (int k = 0; k < 256; k += 64) wcnt[wave][k + lane] = 0;
    const int64_t q0 = (int64_t)blockIdx.x * kRsTile + wave * kQuarter;
    uint64_t key[kRsRounds];
    uint32_t val[kRsRounds];
#pragma unroll
    for (int r = 0; r < kRsRounds; ++r) {
        const int64_t i = q0 + r * 64 + lane;
        key[r] = i < n ? kin[i] : 0;
        val[r] = (vin && i < n) ? vin[i] : 0u;
    }
    const uint64_t lt_mask = (lane == 0) ? 0ULL : (~0ULL >> (64 - lane));
    int dg[kRsRounds], at[kRsRounds];
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kRsRounds; ++r) {
        const bool valid = q0 + r * 64 + lane < n;
        const int d = (int)((key[r] >> shift) & 255);
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const uint64_t m = __ballot(valid && ((d >> b) & 1));
            peers &= ((d >> b) & 1) ? m : ~m;
        }
        const int rank = __popcll(peers & lt_mask);
        const int before = wcnt[wave][d];
        // every lane of the wave has read the count before its leader moves it
        __builtin_amdgcn_wave_barrier();
        if (valid && rank == 0) wcnt[wave][d] = before + __popcll(peers);
        __builtin_amdgcn_wave_barrier();
        dg[r] = valid ? d : -1;
        at[r] = before + rank;
    }
    __syncthreads();
    {
        int c[kRsWaves], tot = 0;
#pragma unroll
        for (int w = 0; w < kRsWaves; ++w) {
            c[w] = wcnt[w][t];
            tot += c[w];
        }
        int all;
        const int lbase = block_excl_scan(tot, wsum, &all);
        goff[t] = offs[t * rs + blockIdx.x] + block_excl_scan(dtot[t], wsum, &all) - lbase;
        int run = lbase;
#pragma unroll
        for (int w = 0; w < kRsWaves; ++w) {
            wcnt[w][t] = run;
            run += c[w];
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kRsRounds; ++r) {
        if (dg[r] >= 0) {
            const int pos = wcnt[wave][dg[r]] + at[r];
            sk[pos] = key[r];
            sv[pos] = val[r];
        }
    }
    __syncthreads();
    const int64_t tile0 = (int64_t)blockIdx.x * kRsTile;
    const int cnt = (int)min((int64_t)kRsTile, n - tile0);
    for (int p = t; p < cnt; p += kRsThreads) {
        const uint64_t k = sk[p];
        const int64_t pos = (int64_t)goff[(int)((k >> shift) & 255)] + p;
        if (pos < 0 || pos >= n) continue;  // unreachable with consistent counts
        if (lo_out) {
            lo_out[pos] = (uint32_t)k;
            hi_out[pos] = (uint32_t)(k >> 32);
        } else {
            kout[pos] = k;
        }
        if (vout) vout[pos] = sv[p];
    }
}

uint64_t* radix_sort_u64_pp(uint64_t* keys, uint32_t* vals, uint64_t* kalt, uint32_t* valt, int64_t n, int bits,
                            hipStream_t s, int begin_bit, uint32_t** vout, uint32_t* lo_out, uint32_t* hi_out) {
    if (vout) *vout = vals;
    if (n <= 1 || bits <= begin_bit) return keys;
    const int nblk = (int)((n + kRsTile - 1) / kRsTile);
    const int rs = (nblk + 3) & ~3;  // histogram row stride: 16-byte aligned rows
    int* hist = (int*)pool_alloc(sizeof(int) * 256 * (size_t)rs);
    int* offs = (int*)pool_alloc(sizeof(int) * 256 * (size_t)rs);
    int* dtot = (int*)pool_alloc(sizeof(int) * 256);
    uint64_t *ka = keys, *kb = kalt;
    uint32_t *va = vals, *vb = vals ? valt : nullptr;
    const int npass = (bits - begin_bit + 7) / 8;
    if (begin_bit + 8 * npass > 64) begin_bit = 64 - 8 * npass;
    for (int pass = 0; pass < npass; ++pass) {
        const int shift = begin_bit + 8 * pass;
        k_rs_hist<<<nblk, kRsThreads, 0, s>>>(ka, n, shift, rs, hist);
        SFMM_LAUNCH_CHECK();
        k_rs_rowscan<<<256, kScanThreads, 0, s>>>(hist, nblk, rs, offs, dtot);
        SFMM_LAUNCH_CHECK();
        const bool last = pass == npass - 1;
        k_rs_scatter<<<nblk, kRsThreads, 0, s>>>(ka, va, kb, vb, n, shift, rs, offs, dtot, last ? lo_out : nullptr,
                                                 last ? hi_out : nullptr);
        SFMM_LAUNCH_CHECK();
        std::swap(ka, kb);
        std::swap(va, vb);
    }
    // freed blocks are only reused by later stream-ordered work on this stream
    pool_free(hist);
    pool_free(offs);
    pool_free(dtot);
    if (vout) *vout = va;
    return ka;
}

void radix_sort_u64(uint64_t* keys, uint32_t* vals, int64_t n, int bits, hipStream_t s, int begin_bit) {
    if (n <= 1 || bits <= begin_bit) return;
    uint64_t* k2 = (uint64_t*)pool_alloc(sizeof(uint64_t) * n);
    uint32_t* v2 = vals ? (uint32_t*)pool_alloc(sizeof(uint32_t) * n) : nullptr;
    uint32_t* vr = nullptr;
    const uint64_t* kr = radix_sort_u64_pp(keys, vals, k2, v2, n, bits, s, begin_bit, &vr);
    if (kr != keys) {  // an odd number of passes leaves the result in the scratch buffers
        SFMM_HIP(hipMemcpyAsync(keys, kr, sizeof(uint64_t) * n, hipMemcpyDeviceToDevice, s));
        if (vals) SFMM_HIP(hipMemcpyAsync(vals, vr, sizeof(uint32_t) * n, hipMemcpyDeviceToDevice, s));
    }
    pool_free(k2);
    if (v2) pool_free(v2);
}

// ------------------------------------------------------------------ sum
__global__ void k_sum_tiles(const double* x, int64_t n, int stride, double* part) {
    __shared__ double sh[256];
    double acc = 0.0;
    for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) acc += x[i * stride];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

void sum_f64(const double* x, int64_t n, double* out, hipStream_t s, int stride) {
    double* part = (double*)pool_alloc(sizeof(double) * 1024);
    k_sum_tiles<<<1024, 256, 0, s>>>(x, n, stride, part);
    SFMM_LAUNCH_CHECK();
    k_sum_tiles<<<1, 256, 0, s>>>(part, 1024, 1, out);
    SFMM_LAUNCH_CHECK();
    pool_free(part);
}

__global__ void k_sum_i64(const long long* x, int64_t n, long long* part) {
    __shared__ long long sh[256];
    long long acc = 0;
    for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) acc += x[i];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

void sum_i64(const long long* x, int64_t n, long long* out, hipStream_t s) {
    long long* part = (long long*)pool_alloc(sizeof(long long) * 1024);
    k_sum_i64<<<1024, 256, 0, s>>>(x, n, part);
    SFMM_LAUNCH_CHECK();
    k_sum_i64<<<1, 256, 0, s>>>(part, 1024, out);
    SFMM_LAUNCH_CHECK();
    pool_free(part);
}

}  // namespace sfmm
