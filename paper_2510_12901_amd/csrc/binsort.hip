// binsort.hip -- tile binning and depth sort.
//
// Order of work (all device, one HIP stream):
//   1. stable LSD radix sort of the particles by their float32 depth key (4 x 8-bit passes);
//   2. super-tile counts (8 x 8-tile blocks touched by the particle's tile rect) gathered in
//      depth order, exclusive scan (uint64) -> pair offsets, total P;
//   3. (super-tile, particle) pairs emitted in depth order, a fixed run of pairs per
//      workgroup (prefix offsets + binary search, so a particle touching many super-tiles is
//      spread over many lanes and the work is even however the pairs cluster);
//   4. stable LSD radix sort of the pairs by super-tile id (one 8-bit pass up to 256
//      super-tiles).
// Sorting by depth first and then stably by super-tile gives (super-tile, depth, index)
// order.  Filtering a super-tile list by "rect contains tile" keeps that order, so every
// tile's exact (depth, index)-ordered list is recovered on chip by the consumer.  Binning
// per 8 x 8 tiles instead of per tile cuts the pairs that go through HBM by ~40x on the
// 1920x1080 camera workloads (large near particles touch hundreds of tiles).
#include "ut_internal.hpp"

namespace ut {

// ---------------------------------------------------------------------------------- fills
namespace {
template <typename T>
__global__ void k_fill(T* p, T v, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}
template <typename T>
hipError_t fill(T* p, T v, size_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const size_t blocks = std::min<size_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_fill<T>, dim3((unsigned)blocks), dim3(256), 0, st, p, v, n);
  return hipGetLastError();
}
}  // namespace

hipError_t fill_u32(uint32_t* p, uint32_t v, size_t n, hipStream_t st) { return fill(p, v, n, st); }
hipError_t fill_u64(uint64_t* p, uint64_t v, size_t n, hipStream_t st) { return fill(p, v, n, st); }
hipError_t fill_f64(double* p, double v, size_t n, hipStream_t st) { return fill(p, v, n, st); }

namespace {

// 32/64-bit lane shuffles (uint64_t is unsigned long here; HIP overloads take long long)
__device__ __forceinline__ uint32_t shfl_up_t(uint32_t x, int d) { return __shfl_up(x, d); }
__device__ __forceinline__ uint64_t shfl_up_t(uint64_t x, int d) {
  return (uint64_t)__shfl_up((unsigned long long)x, d);
}

// ---------------------------------------------------------------------------------- scan
constexpr int kScanThreads = 256;
constexpr int kScanItems = 4;
constexpr int kScanTile = kScanThreads * kScanItems;

// exclusive scan of one value per thread across a THREADS-thread block (sh: THREADS / 64
// words); returns the block total
template <typename T, int THREADS = kScanThreads>
__device__ __forceinline__ T block_exclusive(T v, T* sh, T& total) {
  const int lane = __lane_id(), wave = threadIdx.x >> 6;
  T x = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const T y = shfl_up_t(x, off);
    if (lane >= off) x += y;
  }
  if (lane == 63) sh[wave] = x;
  __syncthreads();
  T before = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < THREADS / 64; ++w) {
    const T s = sh[w];
    if (w < wave) before += s;
    tot += s;
  }
  __syncthreads();
  total = tot;
  return before + x - v;
}

// ---------------------------------------------------------------------------------- radix
constexpr int kRadix = 256;
// A pass ranks its tile with 4 wavefronts of 16 keys per lane, one wavefront per SIMD: 512 or
// 1,024 threads rank a tile faster (13.8 and 14.1 against 15.9 us per pass on 214k keys) but
// need 2 or 4 free wavefront slots per SIMD at once, which a CU busy with another sensor's
// compositing frees later, and the multi-sensor frame lost 1-4%.  The first kRadix threads
// own one digit each in the look-back.
constexpr int kSortThreads = 256;
constexpr int kSortItems = 16;      // keys per lane
constexpr int kSortTile = kSortThreads * kSortItems;
constexpr int kMaxPasses = 4;
constexpr int kHistThreads = 256;
constexpr int kHistItems = 4;                          // keys per lane in the histogram kernel
constexpr int kHistTile = kHistThreads * kHistItems;   // keys per histogram workgroup
static_assert(kSortTile % kHistTile == 0, "a sort tile is a whole number of histogram tiles");
// The digit histograms are kept as kHistParts partial copies, workgroup b adding into copy
// b % kHistParts: device-scope atomics from every workgroup on the same 256 words serialise,
// spread over 16 copies they do not.  A pass reads the sum of the copies.
constexpr int kHistParts = 16;

// Look-back words: bits 30..31 hold the state, bits 0..29 the count.
constexpr uint32_t kLbAggregate = 1u << 30;   // the tile's own digit count is published
constexpr uint32_t kLbPrefix = 2u << 30;      // the inclusive prefix over tiles 0..t is published
constexpr uint32_t kLbCount = (1u << 30) - 1u;

// Digit histograms of every pass in one read of the keys: one workgroup per kHistTile keys
// (a quarter of a sort tile, so four times the workgroups of a pass share the latency), every
// lane's loads issued up front.  Depth keys concentrate in a few high-byte values, so lanes
// are first grouped by equal digit (8 ballots) and only one lane per group adds the group's
// size to the LDS counter; one global atomic per digit present follows.
__global__ __launch_bounds__(kHistThreads) void k_digit_hist(const uint32_t* __restrict__ keys, size_t n_max,
                                                              const uint32_t* __restrict__ n_dev, int passes,
                                                              uint32_t* __restrict__ hist, uint32_t* __restrict__ look,
                                                              size_t look_tiles) {
  __shared__ uint32_t h[kMaxPasses][kRadix];
  const size_t n = n_dev ? (size_t)*n_dev : n_max;
  const size_t start = (size_t)blockIdx.x * kHistTile;
  if (start >= n) return;
  const int lane = __lane_id(), wave = threadIdx.x >> 6;
  // the first workgroup of a sort tile clears the tile's look-back words of every pass (the
  // passes run after this kernel)
  constexpr int kPerTile = kSortTile / kHistTile;
  if (blockIdx.x % kPerTile == 0)
    for (int p = 0; p < passes; ++p)
      look[((size_t)p * look_tiles + blockIdx.x / kPerTile) * kRadix + threadIdx.x] = 0u;
  for (int i = threadIdx.x; i < kMaxPasses * kRadix; i += kHistThreads) (&h[0][0])[i] = 0;
  __syncthreads();
  const size_t base = start + (size_t)wave * (kHistItems * 64) + lane;
  uint32_t key[kHistItems];
#pragma unroll
  for (int k = 0; k < kHistItems; ++k) {
    const size_t i = base + (size_t)k * 64;
    key[k] = i < n ? keys[i] : 0u;
  }
#pragma unroll
  for (int k = 0; k < kHistItems; ++k) {
    const bool valid = base + (size_t)k * 64 < n;
    for (int p = 0; p < passes; ++p) {
      const uint32_t d = (key[k] >> (8 * p)) & (kRadix - 1);
      unsigned long long peers = __ballot(valid);
#pragma unroll
      for (int b = 0; b < 8; ++b) {
        const bool bit = (d >> b) & 1u;
        const unsigned long long m = __ballot(bit);
        peers &= bit ? m : ~m;
      }
      if (valid && (peers >> lane) == 1ull) atomicAdd(&h[p][d], (uint32_t)__popcll(peers));
    }
  }
  __syncthreads();
  uint32_t* part = hist + (size_t)(blockIdx.x % kHistParts) * kMaxPasses * kRadix;
  for (int i = threadIdx.x; i < passes * kRadix; i += kHistThreads) {
    const uint32_t c = (&h[0][0])[i];
    if (c) atomicAdd(&part[i], c);
  }
}

// One stable pass by digit (key >> shift) & 255 with decoupled look-back (single kernel per
// pass).  A look-back word carries its state and count together, so relaxed device-scope
// atomics suffice (an acquire would invalidate the XCD's L2 on every poll).  Workgroups take
// tiles of kSortTile keys in launch order from a ticket counter, so every tile a workgroup
// waits on belongs to a workgroup that is already running and publishes its own digit counts
// before it waits on anything: the waits always end.  Inside a tile, wave w owns keys
// [w*1024, (w+1)*1024) in the order (item, lane); a lane's rank among equal digits of its
// wave comes from 8 ballots (peer mask) plus the wave's running digit count in LDS.  The
// tile is then reordered by digit in LDS so that the global writes form one contiguous run
// per digit.
__global__ __launch_bounds__(kSortThreads) void k_onesweep(const uint32_t* __restrict__ kin,
                                                           const uint32_t* __restrict__ vin,
                                                           uint32_t* __restrict__ kout, uint32_t* __restrict__ vout,
                                                           size_t n_max, const uint32_t* __restrict__ n_dev, int shift,
                                                           const uint32_t* __restrict__ digit_count,
                                                           uint32_t* __restrict__ look, uint32_t* __restrict__ ticket) {
  constexpr int kWaves = kSortThreads / 64;
  __shared__ uint32_t s_tile;
  __shared__ uint32_t wcnt[kWaves][kRadix];
  __shared__ uint32_t local_start[kRadix];   // tile-local exclusive prefix over digits
  __shared__ uint32_t dst_shift[kRadix];     // global start of digit d minus its local start
  __shared__ uint32_t sk[kSortTile], sv[kSortTile];
  __shared__ uint32_t scan_sh[kWaves];
  // The loads that do not depend on the tile (the key count, this thread's digit count) go
  // out together with the ticket, and the tile's keys before the digit-count scan, so the
  // pass waits on two memory round trips before ranking instead of four.
  const size_t n = n_dev ? (size_t)*n_dev : n_max;
  uint32_t c = 0;
  if (threadIdx.x < kRadix) {
#pragma unroll
    for (int g = 0; g < kHistParts; ++g) c += digit_count[(size_t)g * kMaxPasses * kRadix + threadIdx.x];
  }
  if (threadIdx.x == 0) s_tile = atomicAdd(ticket, 1u);
  for (int i = threadIdx.x; i < kWaves * kRadix; i += kSortThreads) (&wcnt[0][0])[i] = 0;
  __syncthreads();
  const uint32_t tile = s_tile;
  const size_t n_tiles = (n + kSortTile - 1) / kSortTile;
  if (tile >= n_tiles) return;
  const int lane = __lane_id(), wave = threadIdx.x >> 6;
  const unsigned long long lt = (1ull << lane) - 1ull;
  const size_t tile0 = (size_t)tile * kSortTile;
  const size_t base = tile0 + (size_t)wave * (kSortItems * 64) + lane;
  const uint32_t tile_n = (uint32_t)std::min<size_t>(kSortTile, n - tile0);
  uint32_t key[kSortItems], val[kSortItems], rank[kSortItems];
#pragma unroll
  for (int k = 0; k < kSortItems; ++k) {
    const size_t i = base + (size_t)k * 64;
    key[k] = i < n ? kin[i] : 0u;
    val[k] = i < n ? vin[i] : 0u;
  }
  // global start of this thread's digit: exclusive prefix of the pass's digit counts
  uint32_t digit_base;
  {
    uint32_t all;
    digit_base = block_exclusive<uint32_t, kSortThreads>(c, scan_sh, all);
  }
#pragma unroll
  for (int k = 0; k < kSortItems; ++k) {
    const bool valid = base + (size_t)k * 64 < n;
    const uint32_t d = (key[k] >> shift) & (kRadix - 1);
    unsigned long long peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1u;
      const unsigned long long m = __ballot(bit);
      peers &= bit ? m : ~m;
    }
    uint32_t r = 0;
    if (valid) r = wcnt[wave][d] + (uint32_t)__popcll(peers & lt);
    rank[k] = r;
    // the highest lane of each peer group advances the wave's count for that digit (the
    // reads above complete first: one wavefront's LDS operations stay in program order)
    if (valid && (peers >> lane) == 1ull) wcnt[wave][d] += (uint32_t)__popcll(peers);
  }
  __syncthreads();

  // thread d < kRadix: the tile's count of digit d, each wave's offset, the tile-local digit
  // start and the look-back for the digit's global start
  {
    const int d = threadIdx.x;
    const bool own = d < kRadix;
    uint32_t total = 0;
    uint32_t* my = look + (size_t)tile * kRadix + d;
    if (own) {
#pragma unroll
      for (int w = 0; w < kWaves; ++w) {
        const uint32_t c = wcnt[w][d];
        wcnt[w][d] = total;
        total += c;
      }
      __hip_atomic_store(my, (tile == 0 ? kLbPrefix : kLbAggregate) | total, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
    }
    uint32_t tile_total;
    const uint32_t lstart = block_exclusive<uint32_t, kSortThreads>(total, scan_sh, tile_total);
    if (own) {
      local_start[d] = lstart;
      uint32_t excl = 0;
      if (tile > 0) {
        // walk back over the predecessors kLookWindow at a time (independent loads in flight),
        // adding aggregates until a published inclusive prefix; tile 0 always publishes one
        constexpr int kLookWindow = 8;
        int64_t j = (int64_t)tile - 1;
        for (;;) {
          uint32_t v[kLookWindow];
#pragma unroll
          for (int q = 0; q < kLookWindow; ++q)
            v[q] = j - q >= 0 ? __hip_atomic_load(look + (size_t)(j - q) * kRadix + d, __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_AGENT)
                              : kLbPrefix;
          int used = 0;
          bool found = false;
#pragma unroll
          for (int q = 0; q < kLookWindow; ++q) {
            if (found || used < q) continue;   // stop at the first prefix or the first gap
            const uint32_t st = v[q] & ~kLbCount;
            if (st == 0u) continue;
            excl += v[q] & kLbCount;
            used = q + 1;
            found = st == kLbPrefix;
          }
          if (found) break;
          j -= used;
          if (used == 0) __builtin_amdgcn_s_sleep(1);
        }
        __hip_atomic_store(my, kLbPrefix | (excl + total), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      dst_shift[d] = digit_base + excl - lstart;
    }
  }
  __syncthreads();
  // reorder the tile by digit in LDS ...
#pragma unroll
  for (int k = 0; k < kSortItems; ++k) {
    if (base + (size_t)k * 64 < n) {
      const uint32_t d = (key[k] >> shift) & (kRadix - 1);
      const uint32_t lp = local_start[d] + wcnt[wave][d] + rank[k];
      sk[lp] = key[k];
      sv[lp] = val[k];
    }
  }
  __syncthreads();
  // ... and write it out: consecutive local positions of one digit go to consecutive addresses
  for (uint32_t lp = threadIdx.x; lp < tile_n; lp += kSortThreads) {
    const uint32_t k = sk[lp];
    const uint32_t dst = dst_shift[(k >> shift) & (kRadix - 1)] + lp;
    kout[dst] = k;
    vout[dst] = sv[lp];
  }
}

}  // namespace

// Bytes of the sort's own workspace for up to n_max keys: per-pass digit counts and tickets
// (radix_clear_words() words at the start, which must be zero when a sort starts), then the
// per-pass look-back words, which the histogram kernel clears per tile.
size_t radix_tiles(size_t n_max) { return (std::max<size_t>(n_max, 1) + kSortTile - 1) / kSortTile; }
size_t radix_ws_bytes(size_t n_max) {
  return 4 * (radix_clear_words() + (size_t)kMaxPasses * radix_tiles(n_max) * kRadix);
}
size_t radix_clear_words() { return (size_t)kHistParts * kMaxPasses * kRadix + kMaxPasses; }

// Sorts (k, v) pairs by the low `bits` bits of k (bits <= 32), stable.  n_max sizes the grid;
// when n_dev is given the kernels read the actual length from it.  Buffers ping-pong;
// *k_res / *v_res receive the buffers holding the result.  `ws` holds radix_ws_bytes(n_max);
// ws_clear: its first radix_clear_words() words are already zero (a kernel before the sort on
// the same stream cleared them), else a fill kernel clears them.
hipError_t radix_sort(uint32_t* kA, uint32_t* kB, uint32_t* vA, uint32_t* vB, size_t n_max,
                      const uint32_t* n_dev, int bits, uint32_t* ws, hipStream_t st,
                      uint32_t** k_res, uint32_t** v_res, bool ws_clear) {
  *k_res = kA;
  *v_res = vA;
  if (n_max == 0 || bits <= 0) return hipSuccess;
  if (n_max > kLbCount || bits > 8 * kMaxPasses) return hipErrorInvalidValue;   // look-back counts are 30-bit
  const int passes = (bits + 7) / 8;
  const size_t tiles = radix_tiles(n_max);
  uint32_t* hist = ws;
  uint32_t* tickets = ws + (size_t)kHistParts * kMaxPasses * kRadix;
  uint32_t* look = tickets + kMaxPasses;
  if (!ws_clear) {
    const hipError_t e = fill_u32(ws, 0u, radix_clear_words(), st);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_digit_hist, dim3((unsigned)((n_max + kHistTile - 1) / kHistTile)), dim3(kHistThreads), 0, st,
                     kA, n_max, n_dev, passes, hist, look, tiles);
  for (int p = 0; p < passes; ++p) {
    hipLaunchKernelGGL(k_onesweep, dim3((unsigned)tiles), dim3(kSortThreads), 0, st, kA, vA, kB, vB, n_max, n_dev,
                       8 * p, hist + p * kRadix, look + (size_t)p * tiles * kRadix, tickets + p);
    std::swap(kA, kB);
    std::swap(vA, vB);
  }
  *k_res = kA;
  *v_res = vA;
  return hipGetLastError();
}

namespace {

int radix_passes(int bits) { return (bits + 7) / 8; }

// ---------------------------------------------------------------------------------- binning
// super-tile columns touched by tile columns [x0, x1] (x1 may pass tiles_x - 1 for a LiDAR
// rect that wraps through azimuth 0); *sx0 receives the first column, columns wrap mod SX
__device__ __forceinline__ int super_cols(int x0, int x1, int tiles_x, int SX, int wrap, int* sx0) {
  if (!wrap || x1 < tiles_x) {
    *sx0 = x0 / kSuper;
    return x1 / kSuper - x0 / kSuper + 1;
  }
  const int nc = (SX - x0 / kSuper) + ((x1 - tiles_x) / kSuper + 1);
  if (nc >= SX) {
    *sx0 = 0;
    return SX;
  }
  *sx0 = x0 / kSuper;
  return nc;
}

// super-tile count of particle i (0 when its tile count is 0)
__device__ __forceinline__ uint32_t super_count(const uint32_t* __restrict__ count, const int32_t* __restrict__ rect,
                                                int n, int i, int tiles_x, int SX, int SH, int wrap) {
  if (!count[i]) return 0u;
  int sx0;
  const int nc = super_cols(rect[i], rect[2 * n + i], tiles_x, SX, wrap, &sx0);
  const int nr = rect[3 * n + i] / SH - rect[n + i] / SH + 1;
  return (uint32_t)(nc * nr);
}

// Offset of block b from the per-block sums of a first pass: every block adds up its
// predecessors' sums itself (a few thousand words at most, from L2), so no scan kernel runs
// between the two passes.  For block 0, *all receives the sum over all nb blocks.
template <typename T>
__device__ __forceinline__ T block_offset(const T* __restrict__ sums, int b, int nb, T* sh /*[4]*/, T& all) {
  const int upto = b == 0 ? nb : b;   // block 0 adds up everything (its own offset is 0)
  T acc = 0;
  for (int i = threadIdx.x; i < upto; i += kScanThreads) acc += sums[i];
  T sum;
  block_exclusive<T>(acc, sh, sum);
  all = sum;
  return b == 0 ? (T)0 : sum;
}

// Visible-particle compaction, pass 1 of 2: per particle its super-tile count (kept for the
// pair emission), per block of kScanTile particles the number of visible ones.  The blocks
// also clear the depth sort's counters (the sort runs after pass 2 on the same stream).
__global__ __launch_bounds__(kScanThreads) void k_prep_reduce(const uint32_t* __restrict__ count,
                                                              const int32_t* __restrict__ rect, int tiles_x, int SX,
                                                              int SH, int wrap, uint32_t* __restrict__ scount, int n,
                                                              uint32_t* __restrict__ sums, uint32_t* __restrict__ clear,
                                                              int n_clear) {
  __shared__ uint32_t sh[4];
  for (int i = blockIdx.x * kScanThreads + threadIdx.x; i < n_clear; i += gridDim.x * kScanThreads) clear[i] = 0u;
  const int base = blockIdx.x * kScanTile + threadIdx.x * kScanItems;
  uint32_t f = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int i = base + k;
    if (i < n) {
      const uint32_t c = super_count(count, rect, n, i, tiles_x, SX, SH, wrap);
      scount[i] = c;
      f += c ? 1u : 0u;
    }
  }
  uint32_t total;
  block_exclusive<uint32_t>(f, sh, total);
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// Pass 2 of 2: the stable compaction, (depth key, index) of the visible particles in index
// order, and *m_dev = their number (block 0).
__global__ __launch_bounds__(kScanThreads) void k_compact_apply(const uint32_t* __restrict__ key,
                                                                const uint32_t* __restrict__ scount, int n,
                                                                const uint32_t* __restrict__ sums, int nb,
                                                                uint32_t* __restrict__ dk, uint32_t* __restrict__ dv,
                                                                uint32_t* __restrict__ m_dev) {
  __shared__ uint32_t sh[4];
  const int base = blockIdx.x * kScanTile + threadIdx.x * kScanItems;
  uint32_t v[kScanItems];
  uint32_t f = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    v[k] = base + k < n && scount[base + k] ? 1u : 0u;
    f += v[k];
  }
  uint32_t all;
  const uint32_t off = block_offset<uint32_t>(sums, blockIdx.x, nb, sh, all);
  if (blockIdx.x == 0 && threadIdx.x == 0) *m_dev = all;
  uint32_t total;
  uint32_t p = block_exclusive<uint32_t>(f, sh, total) + off;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    if (v[k]) {
      dk[p] = key[base + k];
      dv[p] = (uint32_t)(base + k);
      ++p;
    }
  }
}

// Pair offsets, pass 1 of 2: per block of kScanTile depth-ordered particles, the sum of their
// super-tile counts (0 past the visible count).
__global__ __launch_bounds__(kScanThreads) void k_gather_reduce(const uint32_t* __restrict__ order,
                                                                const uint32_t* __restrict__ scount,
                                                                const uint32_t* __restrict__ m_dev, int n,
                                                                uint64_t* __restrict__ sums) {
  __shared__ uint64_t sh[4];
  const int base = blockIdx.x * kScanTile + threadIdx.x * kScanItems;
  const uint32_t m = *m_dev;
  uint64_t t = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k)
    if (base + k < n && (uint32_t)(base + k) < m) t += scount[order[base + k]];
  uint64_t total;
  block_exclusive<uint64_t>(t, sh, total);
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// Pass 2 of 2: offs[i] = exclusive prefix of the super-tile counts in depth order, *total the
// pair total (block 0).
__global__ __launch_bounds__(kScanThreads) void k_gather_apply(const uint32_t* __restrict__ order,
                                                               const uint32_t* __restrict__ scount,
                                                               const uint32_t* __restrict__ m_dev, int n,
                                                               const uint64_t* __restrict__ sums, int nb,
                                                               uint64_t* __restrict__ offs,
                                                               uint64_t* __restrict__ total_out) {
  __shared__ uint64_t sh[4];
  const int base = blockIdx.x * kScanTile + threadIdx.x * kScanItems;
  const uint32_t m = *m_dev;
  uint64_t v[kScanItems];
  uint64_t t = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    v[k] = base + k < n && (uint32_t)(base + k) < m ? (uint64_t)scount[order[base + k]] : 0ull;
    t += v[k];
  }
  uint64_t all;
  const uint64_t off = block_offset<uint64_t>(sums, blockIdx.x, nb, sh, all);
  if (blockIdx.x == 0 && threadIdx.x == 0) *total_out = all;
  uint64_t total;
  uint64_t run = block_exclusive<uint64_t>(t, sh, total) + off;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    if (base + k < n) offs[base + k] = run;
    run += v[k];
  }
}

// ---------------------------------------------------------------------------------- small sets
// Up to kSmallMax particles the whole count stage, and up to kSmallMax pairs the whole pair
// sort, run in one workgroup out of LDS: one launch instead of a chain of short launches that
// each cost more than the work.  The orders are the same: a stable sort by key equals an
// ascending sort of (key, position) words, which a bitonic network gives exactly.
constexpr int kSmallThreads = 1024;
constexpr int kSmallItems = 4;
constexpr int kSmallMax = kSmallThreads * kSmallItems;

// exclusive scan of one value per thread across a kSmallThreads block; returns the total
template <typename T>
__device__ __forceinline__ T small_exclusive(T v, T* sh /*[kSmallThreads / 64]*/, T& total) {
  const int lane = __lane_id(), wave = threadIdx.x >> 6;
  T x = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const T y = shfl_up_t(x, off);
    if (lane >= off) x += y;
  }
  if (lane == 63) sh[wave] = x;
  __syncthreads();
  T before = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < kSmallThreads / 64; ++w) {
    const T s = sh[w];
    if (w < wave) before += s;
    tot += s;
  }
  __syncthreads();
  total = tot;
  return before + x - v;
}

__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t x, int m) {
  return (uint64_t)__shfl_xor((unsigned long long)x, m);
}

// One compare-exchange step of a bitonic network for element e holding a, partner e ^ j
// holding b, in a block of k elements: the lower element keeps the smaller word when the
// block ascends ((e & k) == 0), the larger one otherwise.
__device__ __forceinline__ uint64_t bitonic_keep(uint64_t a, uint64_t b, int e, int j, int k) {
  const bool keep_min = ((e & j) == 0) == ((e & k) == 0);
  return keep_min ? (a < b ? a : b) : (a < b ? b : a);
}

// Bitonic network over the elements e = r * kSmallThreads + threadIdx.x held in v[r]: sorts
// every aligned block of len elements ascending (len a power of two, 64 <= len <= R *
// kSmallThreads).  Partners within a wavefront (distance < 64) are exchanged by lane shuffles,
// across wavefronts through the LDS buffer x (R * kSmallThreads words), within a thread
// between registers.
template <int R>
__device__ void small_bitonic_regs(uint64_t (&v)[R], int len, uint64_t* x) {
  const int t = threadIdx.x;
  for (int k = 2; k <= len; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      if (j < 64) {
#pragma unroll
        for (int r = 0; r < R; ++r) v[r] = bitonic_keep(v[r], shfl_xor_u64(v[r], j), r * kSmallThreads + t, j, k);
      } else if (j < kSmallThreads) {
#pragma unroll
        for (int r = 0; r < R; ++r) x[r * kSmallThreads + t] = v[r];
        __syncthreads();
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const int e = r * kSmallThreads + t;
          v[r] = bitonic_keep(v[r], x[e ^ j], e, j, k);
        }
        __syncthreads();
      } else {
#pragma unroll
        for (int sr = 1; sr < R; sr <<= 1) {
          if (j != sr * kSmallThreads) continue;
#pragma unroll
          for (int r = 0; r < R; ++r) {
            if (r & sr) continue;
            const int e = r * kSmallThreads + t;
            const uint64_t lo = v[r], hi = v[r + sr];
            v[r] = bitonic_keep(lo, hi, e, j, k);
            v[r + sr] = bitonic_keep(hi, lo, e + j, j, k);
          }
        }
      }
    }
  }
}

template <int R>
__device__ void small_sort_lds_r(uint64_t* s, int m, int len) {
  uint64_t v[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int e = r * kSmallThreads + (int)threadIdx.x;
    v[r] = e < m ? s[e] : ~0ull;
  }
  __syncthreads();
  small_bitonic_regs<R>(v, len, s);
#pragma unroll
  for (int r = 0; r < R; ++r) s[r * kSmallThreads + threadIdx.x] = v[r];
  __syncthreads();
}

// Ascending sort of the m <= kSmallMax words s[0, m) in LDS (all threads call it after a
// barrier that follows the writes to s; s holds kSmallMax words).
__device__ void small_sort_lds(uint64_t* s, int m) {
  int len = 64;
  while (len < m) len <<= 1;
  if (len <= kSmallThreads) small_sort_lds_r<1>(s, m, len);
  else if (len <= 2 * kSmallThreads) small_sort_lds_r<2>(s, m, len);
  else small_sort_lds_r<4>(s, m, len);
}

// The count stage of up to kSmallMax particles in one workgroup: super-tile counts, the
// visible particles in (depth key, index) order (dk / dv, *m_dev of them), the exclusive
// prefix of their super-tile counts in that order (offs[j], the total past the visible ones)
// and the total pair count.  Same results as the multi-kernel chain.
__global__ __launch_bounds__(kSmallThreads) void k_count_small(const uint32_t* __restrict__ count,
                                                               const int32_t* __restrict__ rect,
                                                               const uint32_t* __restrict__ key, int n, int tiles_x,
                                                               int SX, int SH, int wrap, uint32_t* __restrict__ scount,
                                                               uint32_t* __restrict__ dk, uint32_t* __restrict__ dv,
                                                               uint32_t* __restrict__ m_dev, uint64_t* __restrict__ offs,
                                                               uint64_t* __restrict__ total) {
  __shared__ uint64_t s_kv[kSmallMax];
  __shared__ uint32_t s_cnt[kSmallMax];
  __shared__ uint64_t s_sum[kSmallThreads / 64];
  const int t = threadIdx.x;
  const int base = t * kSmallItems;
  uint32_t c[kSmallItems];
  uint32_t f = 0;
#pragma unroll
  for (int k = 0; k < kSmallItems; ++k) {
    const int i = base + k;
    c[k] = i < n ? super_count(count, rect, n, i, tiles_x, SX, SH, wrap) : 0u;
    if (i < n) {
      scount[i] = c[k];
      s_cnt[i] = c[k];
    }
    f += c[k] ? 1u : 0u;
  }
  uint64_t m64;
  uint32_t p = (uint32_t)small_exclusive<uint64_t>(f, s_sum, m64);
  const int m = (int)m64;
#pragma unroll
  for (int k = 0; k < kSmallItems; ++k)
    if (c[k]) s_kv[p++] = ((uint64_t)key[base + k] << 32) | (uint32_t)(base + k);
  __syncthreads();
  small_sort_lds(s_kv, m);
  uint64_t v[kSmallItems];
  uint64_t run = 0;
#pragma unroll
  for (int k = 0; k < kSmallItems; ++k) {
    const int j = base + k;
    v[k] = 0;
    if (j < m) {
      const uint64_t w = s_kv[j];
      dk[j] = (uint32_t)(w >> 32);
      dv[j] = (uint32_t)w;
      v[k] = s_cnt[(uint32_t)w];
    }
    run += v[k];
  }
  uint64_t tot;
  run = small_exclusive<uint64_t>(run, s_sum, tot);
#pragma unroll
  for (int k = 0; k < kSmallItems; ++k) {
    if (base + k < n) offs[base + k] = run;
    run += v[k];
  }
  if (t == 0) {
    *m_dev = (uint32_t)m;
    *total = tot;
  }
}

// The pair emission and super-tile sort of up to kSmallMax pairs in one workgroup, for up to
// kSmallMax super-tiles: pairs of the depth-ordered particles ordered by (super-tile, pair
// position), bins.gauss and the per-super-tile [start, end) ranges (0, 0 when empty).  With
// total_dev (device count) the pair count is read there and checked against max_pairs: over
// it nothing is emitted and *overflow is raised.
__global__ __launch_bounds__(kSmallThreads) void k_pairs_small(const uint32_t* __restrict__ order,
                                                               const uint64_t* __restrict__ offs,
                                                               const uint32_t* __restrict__ m_dev,
                                                               const uint2* __restrict__ trect, int n, int tiles_x,
                                                               int SX, int SH, int wrap, uint32_t P_host,
                                                               const uint64_t* __restrict__ total_dev,
                                                               uint64_t max_pairs, uint32_t* __restrict__ overflow,
                                                               uint32_t* __restrict__ gauss, uint32_t* __restrict__ ranges,
                                                               int n_super) {
  __shared__ uint64_t s_kv[kSmallMax];
  __shared__ uint32_t s_g[kSmallMax];
  const int t = threadIdx.x;
  for (int i = t; i < 2 * n_super; i += kSmallThreads) ranges[i] = 0u;
  uint32_t P = P_host;
  if (total_dev) {
    const uint64_t T = *total_dev;
    const bool fits = T <= max_pairs && T <= (uint64_t)kSmallMax;   // the second holds by the launch bound
    P = fits ? (uint32_t)T : 0u;
    if (!fits && overflow && t == 0) overflow[0] = 1u;
  }
  const int m = (int)min((uint32_t)n, *m_dev);
  // every visible particle writes its pairs (super-tile id << 32 | pair position) in depth order
  for (int j = t; j < m; j += kSmallThreads) {
    const uint2 r = trect[order[j]];
    const int x0 = (int)(r.x & 0xFFFFu), y0 = (int)(r.x >> 16), x1 = (int)(r.y & 0xFFFFu), y1 = (int)(r.y >> 16);
    int sx0;
    const int nc = super_cols(x0, x1, tiles_x, SX, wrap, &sx0);
    const int sy0 = y0 / SH, nr = y1 / SH - sy0 + 1;
    uint32_t o = (uint32_t)offs[j];
    for (int yy = 0; yy < nr; ++yy)
      for (int xx = 0; xx < nc; ++xx, ++o) {
        int x = sx0 + xx;
        if (x >= SX) x -= SX;
        if (o < P) {
          s_kv[o] = ((uint64_t)(uint32_t)((sy0 + yy) * SX + x) << 32) | o;
          s_g[o] = order[j];
        }
      }
  }
  __syncthreads();
  small_sort_lds(s_kv, (int)P);
  for (int i = t; i < (int)P; i += kSmallThreads) {
    const uint64_t w = s_kv[i];
    const uint32_t st = (uint32_t)(w >> 32);
    gauss[i] = s_g[(uint32_t)w];
    if (i == 0 || (uint32_t)(s_kv[i - 1] >> 32) != st) ranges[st] = (uint32_t)i;
    if (i == (int)P - 1 || (uint32_t)(s_kv[i + 1] >> 32) != st) ranges[n_super + st] = (uint32_t)(i + 1);
  }
}

// Pair emission balanced over the pairs rather than the particles: near particles touch the
// most super-tiles and sit together in depth order, so emitting per particle leaves a few
// wavefronts with most of the pairs.  Block b writes the kEmitChunk pairs [b C, (b + 1) C):
// two wavefronts find the particles holding its first and last pair (64-way searches of the
// strictly increasing offsets), the block stages those particles' offsets and super-tile
// rects in LDS, and every thread places its pairs by a binary search there.
constexpr int kEmitThreads = 256;
constexpr int kEmitChunk = 1024;

// Largest j in [0, m) with offs[j] <= q, for offs strictly increasing with offs[0] = 0 <= q;
// one wavefront, every lane returns the same j.
__device__ int find_particle(const uint64_t* __restrict__ offs, int m, uint64_t q) {
  const int lane = __lane_id();
  int lo = 0, hi = m;
  while (hi - lo > 1) {
    const int stride = (hi - lo + 63) / 64;
    const int idx = lo + lane * stride;
    const unsigned long long b = __ballot(idx < hi && offs[idx] <= q);
    lo += (63 - __clzll(b)) * stride;   // lane 0 always holds: offs[lo] <= q
    hi = min(hi, lo + stride);
  }
  return lo;
}

__global__ __launch_bounds__(kEmitThreads) void k_emit_pairs(const uint32_t* __restrict__ order,
                                                              const uint64_t* __restrict__ offs,
                                                              const uint32_t* __restrict__ m_dev,
                                                              const uint2* __restrict__ trect, int n, int tiles_x, int SX,
                                                              int SH, int wrap, uint64_t P_host,
                                                              const uint32_t* __restrict__ P_dev,
                                                              uint32_t* __restrict__ pair_key,
                                                              uint32_t* __restrict__ pair_gauss,
                                                              uint32_t* __restrict__ clear, int n_clear) {
  // the blocks clear the pair sort's counters (the sort runs next on the same stream)
  for (int i = blockIdx.x * kEmitThreads + threadIdx.x; i < n_clear; i += gridDim.x * kEmitThreads) clear[i] = 0u;
  const uint64_t P = P_dev ? (uint64_t)*P_dev : P_host;   // device count: 0 = nothing to emit
  const uint64_t q0 = (uint64_t)blockIdx.x * kEmitChunk;
  if (q0 >= P) return;
  const uint32_t len = (uint32_t)min((uint64_t)kEmitChunk, P - q0);
  const int m = min(n, (int)*m_dev);
  __shared__ int s_j[2];
  __shared__ uint32_t s_start[kEmitChunk], s_g[kEmitChunk];
  __shared__ int s_x0[kEmitChunk], s_y0[kEmitChunk], s_w[kEmitChunk];
  __shared__ uint32_t s_skip;
  const int wave = threadIdx.x >> 6;
  if (wave < 2) {
    const int j = find_particle(offs, m, wave == 0 ? q0 : q0 + len - 1);
    if (__lane_id() == 0) s_j[wave] = j;
  }
  __syncthreads();
  const int j0 = s_j[0], cnt = s_j[1] - j0 + 1;   // every particle after j0 starts inside the chunk: cnt <= C
  for (int k = threadIdx.x; k < cnt; k += kEmitThreads) {
    const uint64_t o = offs[j0 + k];
    s_start[k] = o > q0 ? (uint32_t)(o - q0) : 0u;
    if (k == 0) s_skip = (uint32_t)(q0 - o);   // pairs of the first particle before the chunk
    const uint32_t gi = order[j0 + k];
    const uint2 r = trect[gi];
    const int x0 = (int)(r.x & 0xFFFFu), y0 = (int)(r.x >> 16), x1 = (int)(r.y & 0xFFFFu);
    int sx0;
    s_w[k] = super_cols(x0, x1, tiles_x, SX, wrap, &sx0);
    s_x0[k] = sx0;
    s_y0[k] = y0 / SH;
    s_g[k] = gi;
  }
  __syncthreads();
  int top = 1;
  while (2 * top <= cnt) top <<= 1;
  for (uint32_t l = threadIdx.x; l < len; l += kEmitThreads) {
    int k = 0;
    for (int step = top; step > 0; step >>= 1)
      if (k + step < cnt && s_start[k + step] <= l) k += step;
    const uint32_t q = l - s_start[k] + (k == 0 ? s_skip : 0u);
    const int w = s_w[k];
    const int y = s_y0[k] + (int)(q / (uint32_t)w);
    int x = s_x0[k] + (int)(q % (uint32_t)w);
    if (x >= SX) x -= SX;
    pair_key[q0 + l] = (uint32_t)(y * SX + x);
    pair_gauss[q0 + l] = s_g[k];
  }
}

__global__ void k_ranges(const uint32_t* __restrict__ tiles, uint64_t P_max, const uint32_t* __restrict__ P_dev,
                         uint32_t* __restrict__ ranges, int n_tiles) {
  const uint64_t P = P_dev ? (uint64_t)*P_dev : P_max;
  const uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (i >= P) return;
  const uint32_t t = tiles[i];
  if (i == 0 || tiles[i - 1] != t) ranges[t] = (uint32_t)i;
  if (i == P - 1 || tiles[i + 1] != t) ranges[n_tiles + t] = (uint32_t)(i + 1);
}

// ---------------------------------------------------------------------------------- per-tile lists
// One workgroup per tile scans its super-tile bin; tile_fill compacts the entries whose
// rect contains the tile, in bin order, with one ballot + popcount per wavefront.
__global__ __launch_bounds__(256) void k_tile_count(SensorK s, const uint2* __restrict__ trect,
                                                     const uint32_t* __restrict__ bgauss,
                                                     const uint32_t* __restrict__ branges, int n_super,
                                                     uint32_t* __restrict__ ranges, unsigned long long* total) {
  __shared__ uint32_t wsum[4];
  const int tile = blockIdx.x;
  const int n_tiles = s.tiles_x * s.tiles_y;
  const int tx = tile % s.tiles_x, ty = tile / s.tiles_x;
  const int sid = super_of_tile(tile, s);
  const uint32_t start = branges[sid], end = branges[n_super + sid];
  uint32_t cnt = 0;
  for (uint32_t pos = start + threadIdx.x; pos < end; pos += 256) {
    const bool hit = rect_covers(trect[bgauss[pos]], tx, ty, s);
    cnt += hit ? 1u : 0u;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) cnt += (uint32_t)__shfl_xor(cnt, o);
  if (__lane_id() == 0) wsum[threadIdx.x >> 6] = cnt;
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t t = wsum[0] + wsum[1] + wsum[2] + wsum[3];
    ranges[n_tiles + tile] = t;
    if (t) atomicAdd(total, (unsigned long long)t);
  }
}

// single workgroup: counts (in the end half of ranges) -> [start, end) ranges
__global__ __launch_bounds__(256) void k_tile_scan(uint32_t* ranges, int n_tiles) {
  __shared__ uint32_t sh[4];
  uint32_t carry = 0;
  for (int base = 0; base < n_tiles; base += 256) {
    const int i = base + threadIdx.x;
    const uint32_t c = i < n_tiles ? ranges[n_tiles + i] : 0u;
    uint32_t tot;
    const uint32_t ex = block_exclusive<uint32_t>(c, sh, tot);
    if (i < n_tiles) {
      ranges[i] = carry + ex;
      ranges[n_tiles + i] = carry + ex + c;
    }
    carry += tot;
  }
}

__global__ __launch_bounds__(256) void k_tile_fill(SensorK s, const uint2* __restrict__ trect,
                                                    const uint32_t* __restrict__ bgauss,
                                                    const uint32_t* __restrict__ branges, int n_super,
                                                    const uint32_t* __restrict__ ranges, uint32_t* __restrict__ gauss) {
  __shared__ uint32_t wcnt[4];
  const int tile = blockIdx.x;
  const int tx = tile % s.tiles_x, ty = tile / s.tiles_x;
  const int sid = super_of_tile(tile, s);
  const uint32_t start = branges[sid], end = branges[n_super + sid];
  uint32_t out = ranges[tile];
  const int lane = __lane_id(), wave = threadIdx.x >> 6;
  const unsigned long long lt = (1ull << lane) - 1ull;
  for (uint32_t base = start; base < end; base += 256) {
    const uint32_t pos = base + threadIdx.x;
    uint32_t g = 0;
    bool hit = false;
    if (pos < end) {
      g = bgauss[pos];
      hit = rect_covers(trect[g], tx, ty, s);
    }
    const unsigned long long m = __ballot(hit);
    if (lane == 0) wcnt[wave] = (uint32_t)__popcll(m);
    __syncthreads();
    uint32_t before = 0, total = 0;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      const uint32_t c = wcnt[w];
      if (w < wave) before += c;
      total += c;
    }
    if (hit) gauss[out + before + (uint32_t)__popcll(m & lt)] = g;
    out += total;
    __syncthreads();
  }
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

int tile_bits(int n_tiles) {
  int b = 1;
  while (b < 31 && (1u << b) < (uint32_t)n_tiles) ++b;
  return b;
}

}  // namespace

CountWorkspace count_workspace(void* base, int n) {
  CountWorkspace w;
  char* p = static_cast<char*>(base);
  size_t o = 0;
  auto take = [&](size_t bytes) { char* r = p ? p + o : nullptr; o += align256(bytes); return r; };
  const size_t nn = (size_t)(n > 0 ? n : 1);
  w.dkA = reinterpret_cast<uint32_t*>(take(4 * nn));
  w.dkB = reinterpret_cast<uint32_t*>(take(4 * nn));
  w.dvA = reinterpret_cast<uint32_t*>(take(4 * nn));
  w.dvB = reinterpret_cast<uint32_t*>(take(4 * nn));
  w.offs = reinterpret_cast<uint64_t*>(take(8 * (nn + 1)));
  w.total = reinterpret_cast<uint64_t*>(take(8));
  w.scount = reinterpret_cast<uint32_t*>(take(4 * nn));
  w.m_dev = reinterpret_cast<uint32_t*>(take(4));
  w.hist = reinterpret_cast<uint32_t*>(take(radix_ws_bytes(nn)));
  w.scan_aux = reinterpret_cast<uint64_t*>(take(8 * ((nn + 1 + kScanTile - 1) / kScanTile + 1)));
  w.bytes = o;
  return w;
}

PairWorkspace pair_workspace(void* base, uint64_t n_pairs) {
  PairWorkspace w;
  char* p = static_cast<char*>(base);
  size_t o = 0;
  auto take = [&](size_t bytes) { char* r = p ? p + o : nullptr; o += align256(bytes); return r; };
  const size_t mp = (size_t)(n_pairs > 0 ? n_pairs : 1);
  w.tkA = reinterpret_cast<uint32_t*>(take(4 * mp));
  w.tkB = reinterpret_cast<uint32_t*>(take(4 * mp));
  w.tv = reinterpret_cast<uint32_t*>(take(4 * mp));
  w.hist = reinterpret_cast<uint32_t*>(take(radix_ws_bytes(mp)));
  w.n_dev = reinterpret_cast<uint32_t*>(take(4));
  w.bytes = o;
  return w;
}

hipError_t launch_bin_count(const ut_projected& p, int n, const SensorK& s, CountWorkspace& ws, hipStream_t st) {
  if (n == 0) {
    hipError_t e = fill_u64(ws.total, 0, 1, st);
    if (e == hipSuccess) e = fill_u32(ws.m_dev, 0u, 1, st);
    return e;
  }
  const int nb = (n + kScanTile - 1) / kScanTile;
  const int wrap = s.kind == UT_LIDAR ? 1 : 0;
  if (n <= kSmallMax) {
    hipLaunchKernelGGL(k_count_small, dim3(1), dim3(kSmallThreads), 0, st, p.count, p.rect, p.key, n, s.tiles_x,
                       s.super_x, s.super_h, wrap, ws.scount, ws.dkA, ws.dvA, ws.m_dev, ws.offs, ws.total);
    return hipGetLastError();
  }
  uint32_t* sums32 = reinterpret_cast<uint32_t*>(ws.scan_aux);
  // visible particles (tile count > 0) compacted in index order, then depth-sorted
  hipLaunchKernelGGL(k_prep_reduce, dim3(nb), dim3(kScanThreads), 0, st, p.count, p.rect, s.tiles_x, s.super_x,
                     s.super_h, wrap, ws.scount, n, sums32, ws.hist, (int)radix_clear_words());
  hipLaunchKernelGGL(k_compact_apply, dim3(nb), dim3(kScanThreads), 0, st, p.key, ws.scount, n, sums32, nb, ws.dkA,
                     ws.dvA, ws.m_dev);
  uint32_t *kr, *vr;
  hipError_t e = radix_sort(ws.dkA, ws.dkB, ws.dvA, ws.dvB, (size_t)n, ws.m_dev, 32, ws.hist, st, &kr, &vr, true);
  if (e != hipSuccess) return e;
  // 4 passes: the result is back in the A buffers; the pair offsets in depth order
  hipLaunchKernelGGL(k_gather_reduce, dim3(nb), dim3(kScanThreads), 0, st, ws.dvA, ws.scount, ws.m_dev, n,
                     ws.scan_aux);
  hipLaunchKernelGGL(k_gather_apply, dim3(nb), dim3(kScanThreads), 0, st, ws.dvA, ws.scount, ws.m_dev, n,
                     ws.scan_aux, nb, ws.offs, ws.total);
  return hipGetLastError();
}

hipError_t launch_bin_sort(const ut_projected& p, int n, const SensorK& s, CountWorkspace& ws,
                           PairWorkspace& pw, uint64_t n_pairs, const ut_bin_lists& bins, hipStream_t st) {
  const int n_super = s.super_x * s.super_y;
  hipError_t e = fill_u32(bins.ranges, 0u, 2 * (size_t)n_super, st);
  if (e != hipSuccess || n_pairs == 0 || n == 0) return e;
  if (n_pairs <= (uint64_t)kSmallMax) {
    hipLaunchKernelGGL(k_pairs_small, dim3(1), dim3(kSmallThreads), 0, st, ws.dvA, ws.offs, ws.m_dev,
                       reinterpret_cast<const uint2*>(p.trect), n, s.tiles_x, s.super_x, s.super_h,
                       s.kind == UT_LIDAR ? 1 : 0, (uint32_t)n_pairs, nullptr, 0ull, nullptr, bins.gauss, bins.ranges,
                       n_super);
    return hipGetLastError();
  }
  const int bits = tile_bits(n_super);
  // place the emitted pair values so that the last radix pass writes into bins.gauss
  uint32_t* v_first = (radix_passes(bits) % 2) ? pw.tv : bins.gauss;
  uint32_t* v_second = (radix_passes(bits) % 2) ? bins.gauss : pw.tv;
  const unsigned blocks = (unsigned)((n_pairs + kEmitChunk - 1) / kEmitChunk);
  hipLaunchKernelGGL(k_emit_pairs, dim3(blocks), dim3(kEmitThreads), 0, st, ws.dvA, ws.offs, ws.m_dev,
                     reinterpret_cast<const uint2*>(p.trect), n, s.tiles_x, s.super_x, s.super_h,
                     s.kind == UT_LIDAR ? 1 : 0, n_pairs, nullptr, pw.tkA, v_first, pw.hist, (int)radix_clear_words());
  uint32_t *kr, *vr;
  e = radix_sort(pw.tkA, pw.tkB, v_first, v_second, (size_t)n_pairs, nullptr, bits, pw.hist, st, &kr, &vr, true);
  if (e != hipSuccess) return e;
  const unsigned rb = (unsigned)((n_pairs + 255) / 256);
  hipLaunchKernelGGL(k_ranges, dim3(rb), dim3(256), 0, st, kr, n_pairs, nullptr, bins.ranges, n_super);
  return hipGetLastError();
}

namespace {
// The pair total of the count step against the capacity: the sort's device count is the
// total when it fits, else 0 (nothing is emitted) and the overflow flag is raised.
__global__ void k_pair_guard(const uint64_t* __restrict__ total, uint64_t max_pairs, uint32_t* __restrict__ n_dev,
                             uint32_t* __restrict__ overflow) {
  if (threadIdx.x != 0) return;
  const uint64_t P = *total;
  const bool fits = P <= max_pairs;
  n_dev[0] = fits ? (uint32_t)P : 0u;
  if (!fits && overflow) overflow[0] = 1u;
}
}  // namespace

hipError_t launch_bin_sort_device(const ut_projected& p, int n, const SensorK& s, CountWorkspace& ws,
                                  PairWorkspace& pw, uint64_t max_pairs, const ut_bin_lists& bins,
                                  uint32_t* overflow, hipStream_t st) {
  const int n_super = s.super_x * s.super_y;
  // the pair total is not known here: the one-workgroup sort runs when the capacity, or every
  // particle touching every super-tile, bounds it by kSmallMax
  const uint64_t bound = std::min<uint64_t>(max_pairs, (uint64_t)n * (uint64_t)n_super);
  if (max_pairs > 0 && n > 0 && bound <= (uint64_t)kSmallMax) {
    hipLaunchKernelGGL(k_pairs_small, dim3(1), dim3(kSmallThreads), 0, st, ws.dvA, ws.offs, ws.m_dev,
                       reinterpret_cast<const uint2*>(p.trect), n, s.tiles_x, s.super_x, s.super_h,
                       s.kind == UT_LIDAR ? 1 : 0, 0u, ws.total, max_pairs, overflow, bins.gauss, bins.ranges,
                       n_super);
    return hipGetLastError();
  }
  hipError_t e = fill_u32(bins.ranges, 0u, 2 * (size_t)n_super, st);
  if (e != hipSuccess || max_pairs == 0 || n == 0) return e;
  hipLaunchKernelGGL(k_pair_guard, dim3(1), dim3(64), 0, st, ws.total, max_pairs, pw.n_dev, overflow);
  const int bits = tile_bits(n_super);
  uint32_t* v_first = (radix_passes(bits) % 2) ? pw.tv : bins.gauss;
  uint32_t* v_second = (radix_passes(bits) % 2) ? bins.gauss : pw.tv;
  const unsigned blocks = (unsigned)((max_pairs + kEmitChunk - 1) / kEmitChunk);
  hipLaunchKernelGGL(k_emit_pairs, dim3(blocks), dim3(kEmitThreads), 0, st, ws.dvA, ws.offs, ws.m_dev,
                     reinterpret_cast<const uint2*>(p.trect), n, s.tiles_x, s.super_x, s.super_h,
                     s.kind == UT_LIDAR ? 1 : 0, max_pairs, pw.n_dev, pw.tkA, v_first, pw.hist,
                     (int)radix_clear_words());
  uint32_t *kr, *vr;
  e = radix_sort(pw.tkA, pw.tkB, v_first, v_second, (size_t)max_pairs, pw.n_dev, bits, pw.hist, st, &kr, &vr, true);
  if (e != hipSuccess) return e;
  const unsigned rb = (unsigned)((max_pairs + 255) / 256);
  hipLaunchKernelGGL(k_ranges, dim3(rb), dim3(256), 0, st, kr, max_pairs, pw.n_dev, bins.ranges, n_super);
  return hipGetLastError();
}

hipError_t launch_tile_lists_count(const ut_projected& p, const SensorK& s, const ut_bin_lists& bins,
                                   const ut_tile_lists& lists, hipStream_t st) {
  const int n_tiles = s.tiles_x * s.tiles_y;
  hipError_t e = fill_u64(lists.n_pairs_dev, 0, 1, st);
  if (e != hipSuccess || n_tiles == 0) return e;
  hipLaunchKernelGGL(k_tile_count, dim3(n_tiles), dim3(256), 0, st, s, reinterpret_cast<const uint2*>(p.trect),
                     bins.gauss, bins.ranges, s.super_x * s.super_y, lists.ranges,
                     reinterpret_cast<unsigned long long*>(lists.n_pairs_dev));
  hipLaunchKernelGGL(k_tile_scan, dim3(1), dim3(256), 0, st, lists.ranges, n_tiles);
  return hipGetLastError();
}

hipError_t launch_tile_lists_fill(const ut_projected& p, const SensorK& s, const ut_bin_lists& bins,
                                  const ut_tile_lists& lists, hipStream_t st) {
  const int n_tiles = s.tiles_x * s.tiles_y;
  if (n_tiles == 0) return hipSuccess;
  hipLaunchKernelGGL(k_tile_fill, dim3(n_tiles), dim3(256), 0, st, s, reinterpret_cast<const uint2*>(p.trect),
                     bins.gauss, bins.ranges, s.super_x * s.super_y, lists.ranges, lists.gauss);
  return hipGetLastError();
}

}  // namespace ut
