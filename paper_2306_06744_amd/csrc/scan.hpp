// scan.hpp -- single-pass exclusive scan with decoupled look-back, for
// kernels that count outputs per input and then write them in input order.
//
// Each workgroup takes a tile ticket from a device counter (so every earlier
// tile is already resident), reduces its counts, publishes the aggregate,
// walks back over earlier tiles' published words until it meets an inclusive
// prefix, then publishes its own inclusive prefix.  A tile status word packs
// a 2-bit state (0 not ready, 1 aggregate, 2 inclusive prefix) over a 62-bit
// value.  The status words and the ticket counter must be zero at launch.
// The wait on a predecessor is bounded; on overrun the kernel records
// ERR_LOOKBACK and carries on with a wrong offset so that every wave exits.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lt {

constexpr int kBlock = 256;   // workgroup of the plain kernels
constexpr int kItems = 8;     // items per thread in scan-emit kernels
// Scan-emit kernels over the leaves on the critical path (adapt, balance
// refinement) run 1024-thread tiles of 8192 items: ~1.6M leaves are 200
// tiles, and the look-back of the last one crosses about 4 windows of 64
// predecessors (each window one round trip to device-coherent memory) instead
// of 13.  Short scans (transfer groups) and scans that may run beside another
// stream's kernels (connectivity rows, the split transfer's lists), where a
// 1024-thread workgroup would wait for a whole free CU, keep 256-thread tiles
// of 2048 items.
constexpr int kScanBig = 1024;
constexpr int kScanSmall = kBlock;
constexpr int64_t kTileMax = int64_t(kScanBig) * kItems;
constexpr int64_t kTileMin = int64_t(kScanSmall) * kItems;

enum : unsigned {
  ERR_LOOKBACK = 1u << 0,
  ERR_BAD_FLAG = 1u << 1,
  ERR_UNBALANCED = 1u << 2,
  ERR_INVALID_TREE = 1u << 3,
  ERR_MAP = 1u << 4,
  ERR_CAPACITY = 1u << 5,
  ERR_BALANCE_PASSES = 1u << 6,  // a captured cycle's fixed balance passes did not converge
};

// A number of items known either on the host (p null) or only on the device
// (p points at it; the launch is then sized for the capacity n).
struct Count {
  int64_t n;
  const int64_t* p;
  // captured cycles: the count expected at capture (0: none); a launch may
  // size its grid for it and stride over the rest
  int64_t hint = 0;
  __device__ int64_t get() const { return p ? *p : n; }
};

struct ScanState {
  uint64_t* status;       // one word per tile of the launch
  unsigned long long* ticket;
  unsigned* err;
  int64_t* total;         // written by the last tile: sum of all counts
  Count items;            // items scanned; tiles = max(1, ceil(items / tile))
  int64_t tile;           // items per tile: the kernel's workgroup size times kItems
  int64_t* commit;        // optional (captured cycles): also receives min(total, commit_cap),
  int64_t commit_cap;     // with ERR_CAPACITY raised when the total exceeds it
};

// The last tile's publication of the total (and of its clamped copy).
__device__ inline void publish_total(const ScanState& st, int64_t v) {
  *st.total = v;
  if (st.commit) {
    if (v > st.commit_cap) atomicOr(st.err, ERR_CAPACITY);
    *st.commit = v > st.commit_cap ? st.commit_cap : v;
  }
}

// Tiles that hold items (>= 1).  Launches sized for a capacity have more
// workgroups than this; the extra ones take a ticket and leave at once.
__device__ inline int64_t scan_tiles(const ScanState& st) {
  const int64_t n = st.items.get();
  return n > 0 ? (n + st.tile - 1) / st.tile : 1;
}

constexpr uint64_t kStAgg = uint64_t(1) << 62;
constexpr uint64_t kStInc = uint64_t(2) << 62;
constexpr uint64_t kStVal = (uint64_t(1) << 62) - 1;
constexpr long kSpinLimit = 1L << 20;

// A status word carries its own value, and no tile reads data written by
// another tile of the same launch, so the words need device-coherent access
// but no ordering of other memory: relaxed agent-scope atomics.  (Acquire /
// release at agent scope would write back or invalidate an XCD's whole L2 on
// every publish and every poll.)
__device__ inline uint64_t ld_status(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void st_status(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Inclusive scan of v across the 64 lanes of a wave.
__device__ inline int64_t wave_inclusive(int64_t v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int64_t y = __shfl_up(v, o, 64);
    if (lane >= o) v += y;
  }
  return v;
}

// Exclusive scan of v over a workgroup of BLOCK threads; *total receives the sum.
template <int BLOCK>
__device__ inline int64_t block_exclusive(int64_t v, int64_t* total) {
  constexpr int kWaves = BLOCK / 64;
  __shared__ int64_t wsum[kWaves];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t inc = wave_inclusive(v);
  if (lane == 63) wsum[w] = inc;
  __syncthreads();
  int64_t before = 0, all = 0;
#pragma unroll
  for (int i = 0; i < kWaves; ++i) {
    if (i < w) before += wsum[i];
    all += wsum[i];
  }
  __syncthreads();
  *total = all;
  return before + inc - v;
}

// Appends v entries per lane to a list whose length is *count (one atomic per
// wave); returns this lane's first position.  Every lane of the wave calls it.
__device__ inline int64_t wave_append(int64_t v, int64_t* count) {
  const int64_t inc = wave_inclusive(v);
  const int64_t tot = __shfl(inc, 63, 64);
  int64_t b = 0;
  if ((threadIdx.x & 63) == 63 && tot > 0)
    b = int64_t(atomicAdd(reinterpret_cast<unsigned long long*>(count), (unsigned long long)tot));
  b = __shfl(b, 63, 64);
  return b + inc - v;
}

// Sum of v over the 64 lanes of a wave (result in every lane).
__device__ inline int64_t wave_sum(int64_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Called by every thread of the tile; returns the tile's exclusive prefix.
// The first wave does the look-back: lane k reads the status word of tile
// (base - k), so one round trip covers 64 predecessors.  The window is
// resolved once every lane up to the nearest inclusive prefix is ready;
// if all 64 hold aggregates, their sum is taken and the window moves on.
__device__ inline int64_t tile_prefix(const ScanState& st, int64_t tile, int64_t aggregate) {
  __shared__ int64_t s_prefix;
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    int64_t excl = 0;
    if (tile == 0) {
      if (lane == 0) st_status(&st.status[0], kStInc | uint64_t(aggregate));
    } else {
      if (lane == 0) st_status(&st.status[tile], kStAgg | uint64_t(aggregate));
      int64_t base = tile - 1;
      long spins = 0;
      for (;;) {
        const int64_t idx = base - lane;
        const uint64_t w = idx >= 0 ? ld_status(&st.status[idx]) : (kStInc | 0);
        const uint64_t state = w & ~kStVal;
        const unsigned long long ready = __ballot(state != 0);
        const unsigned long long inc = __ballot(state == kStInc);
        if (inc) {
          const int L = __ffsll(inc) - 1;  // nearest inclusive prefix
          const unsigned long long need = L == 63 ? ~0ull : ((1ull << (L + 1)) - 1);
          if ((ready & need) == need) {
            excl += wave_sum(lane <= L ? int64_t(w & kStVal) : 0);
            break;
          }
        } else if (ready == ~0ull) {
          excl += wave_sum(int64_t(w & kStVal));
          base -= 64;
          continue;
        }
        if (++spins > kSpinLimit) {
          if (lane == 0) atomicOr(st.err, ERR_LOOKBACK);
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
      if (lane == 0) st_status(&st.status[tile], kStInc | uint64_t(excl + aggregate));
    }
    if (lane == 0) {
      if (tile == scan_tiles(st) - 1) publish_total(st, excl + aggregate);
      s_prefix = excl;
    }
  }
  __syncthreads();
  return s_prefix;
}

// Workgroups of a scan launch: one per tile of the (host) item count or capacity.
inline unsigned grid_tiles(const ScanState& st) {
  const int64_t n = st.items.n;
  return unsigned(n > 0 ? (n + st.tile - 1) / st.tile : 1);
}

__device__ inline int64_t take_ticket(const ScanState& st) {
  __shared__ int64_t s_tile;
  if (threadIdx.x == 0) s_tile = int64_t(atomicAdd(st.ticket, 1ull));
  __syncthreads();
  return s_tile;
}

}  // namespace lt
