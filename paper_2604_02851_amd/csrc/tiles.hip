// Tile lists: depth pre-sort of the visible pairs (its first pass takes them
// from the dense (view, Gaussian) arrays, compacting as it sorts), key
// emission, radix sort by tile, per-tile ranges.
//
// Order required by the compositing rule: within a tile, splats ascend by
// (FP32 depth bits, Gaussian index).  Instead of sorting one 64-bit
// (tile | depth) key per (tile, Gaussian) pair, the visible (view, Gaussian)
// pairs (a few per Gaussian) are sorted by depth first, keys are emitted in
// that order, and a stable sort on the tile bits alone finishes the job:
// 4 passes over the visible pairs plus ceil(tile bits / 8) passes over the
// keys, instead of ~7 passes over the keys.
//
// All kernels are driven by device-side counts so the stage can be captured
// in a graph: grids are sized for the plan's capacity and idle blocks exit.
#include "internal.h"

namespace gs {
namespace {

constexpr int B = kSortBlock;
constexpr int NW = B / 64;
static_assert(B == 256, "one thread per radix digit");

__device__ __forceinline__ uint32_t dev_count(const uint32_t* dcount, int64_t max_count) {
  if (!dcount) return (uint32_t)max_count;
  const uint32_t c = *dcount;
  return c < (uint64_t)max_count ? c : (uint32_t)max_count;
}

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  return x;
}

// Exclusive scan over the block (B threads); *total receives the block sum.
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t x, uint32_t* s_wave, uint32_t* total) {
  const uint32_t inc = wave_incl_scan(x);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 63) s_wave[w] = inc;
  __syncthreads();
  uint32_t pre = 0, tot = 0;
#pragma unroll
  for (int k = 0; k < NW; ++k) {
    const uint32_t s = s_wave[k];
    pre += (k < w) ? s : 0u;
    tot += s;
  }
  __syncthreads();
  *total = tot;
  return pre + inc - x;
}

__device__ __forceinline__ uint32_t rect_area(uint2 r) {
  // (tx0 | ty0 << 16, tx1 | ty1 << 16): inclusive tile rectangle
  return ((r.y & 0xffffu) - (r.x & 0xffffu) + 1u) * ((r.y >> 16) - (r.x >> 16) + 1u);
}

// Value source of a scan: a[k], (a[k] != 0), a[idx[k]], or the area of
// tile rectangle k (mode 3, a = rectangles as uint2).
struct ScanSrc {
  const uint32_t* a;
  const uint32_t* idx;
  int mode;
  __device__ __forceinline__ uint32_t operator()(uint32_t k) const {
    if (mode == 0) return a[k];
    if (mode == 1) return a[k] != 0u ? 1u : 0u;
    if (mode == 3) return rect_area(reinterpret_cast<const uint2*>(a)[k]);
    return a[idx[k]];
  }
  // Four consecutive values from k (a multiple of 4) with one 16-byte load of
  // the directly indexed array.
  __device__ __forceinline__ void four(uint32_t k, uint32_t v[4]) const {
    if (mode == 3) {
      const uint4 x = *reinterpret_cast<const uint4*>(a + 2 * (size_t)k);
      const uint4 y = *reinterpret_cast<const uint4*>(a + 2 * (size_t)k + 4);
      v[0] = rect_area(make_uint2(x.x, x.y)), v[1] = rect_area(make_uint2(x.z, x.w));
      v[2] = rect_area(make_uint2(y.x, y.y)), v[3] = rect_area(make_uint2(y.z, y.w));
      return;
    }
    const uint4 x = *reinterpret_cast<const uint4*>((mode == 2 ? idx : a) + k);
    if (mode == 0) {
      v[0] = x.x, v[1] = x.y, v[2] = x.z, v[3] = x.w;
    } else if (mode == 1) {
      v[0] = x.x != 0u, v[1] = x.y != 0u, v[2] = x.z != 0u, v[3] = x.w != 0u;
    } else {
      v[0] = a[x.x], v[1] = a[x.y], v[2] = a[x.z], v[3] = a[x.w];
    }
  }
  __device__ __forceinline__ bool vec_ok() const {
    return ((reinterpret_cast<uintptr_t>(mode == 2 ? idx : a)) & 15u) == 0;
  }
};

// Chunk layout of the scan kernels: thread t holds elements
//   begin + r * 4B + 4t + c   (round r < kRounds, component c < 4),
// so every round is one coalesced 16-byte load per thread.
constexpr int kRounds = kSortItems / 4;
static_assert(kRounds * 4 * B == kSortChunk, "scan chunk layout");

// The uniform choice between the whole-chunk and the ragged form is taken
// once, outside the rounds, so that the whole-chunk form issues all of its
// loads before waiting for any (chosen per round, the two forms' merged
// registers made every round's load wait for the previous one).
__device__ __forceinline__ void load_chunk(const ScanSrc& src, uint64_t begin, uint32_t n,
                                           uint32_t v[kRounds][4]) {
  if (begin + kSortChunk <= n && src.vec_ok()) {
#pragma unroll
    for (int r = 0; r < kRounds; ++r) src.four((uint32_t)(begin + (uint64_t)r * 4 * B + 4u * threadIdx.x), v[r]);
  } else {
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
      const uint64_t k = begin + (uint64_t)r * 4 * B + 4u * threadIdx.x;
#pragma unroll
      for (int c = 0; c < 4; ++c) v[r][c] = k + c < n ? src((uint32_t)(k + c)) : 0u;
    }
  }
}

__global__ __launch_bounds__(B) void k_scan_reduce(ScanSrc src, int64_t max_count, const uint32_t* dcount,
                                                   uint32_t* partial) {
  __shared__ uint32_t s_wave[NW];
  const uint32_t n = dev_count(dcount, max_count);
  const uint64_t begin = (uint64_t)blockIdx.x * kSortChunk;
  if (begin >= n) return;
  uint32_t v[kRounds][4];
  load_chunk(src, begin, n, v);
  uint32_t s = 0;
#pragma unroll
  for (int r = 0; r < kRounds; ++r) s += (v[r][0] + v[r][1]) + (v[r][2] + v[r][3]);
  uint32_t tot;
  block_excl_scan(s, s_wave, &tot);
  if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

// Single block: exclusive scan of the per-chunk partial sums in place.
__global__ __launch_bounds__(1024) void k_scan_partials(int64_t max_count, const uint32_t* dcount, uint32_t* partial,
                                                        uint32_t* total) {
  __shared__ uint32_t s_w[16];
  __shared__ uint32_t s_carry;
  const uint32_t n = dev_count(dcount, max_count);
  const uint32_t np = (uint32_t)((n + kSortChunk - 1) / kSortChunk);
  if (threadIdx.x == 0) s_carry = 0;
  __syncthreads();
  for (uint32_t base = 0; base < np; base += 1024) {
    const uint32_t k = base + threadIdx.x;
    const uint32_t x = k < np ? partial[k] : 0u;
    const uint32_t inc = wave_incl_scan(x);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 63) s_w[w] = inc;
    __syncthreads();
    uint32_t pre = 0, tot = 0;
    for (int q = 0; q < 16; ++q) {
      pre += (q < w) ? s_w[q] : 0u;
      tot += s_w[q];
    }
    const uint32_t carry = s_carry;
    if (k < np) partial[k] = carry + pre + inc - x;
    __syncthreads();
    if (threadIdx.x == 0) s_carry = carry + tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    partial[np] = s_carry;
    if (total) *total = s_carry;
  }
}

// With `firsts` (the key-offset scan), element k, whose run of out[k] .. out[k]
// + value - 1 slots it now knows, also records itself as the owner of every
// chunk of kSortChunk slots that starts inside that run: firsts[m] = k for
// m K in [out[k], out[k] + value), m < firsts_len.
// With `direct`, partial holds the chunks' own sums (k_scan_partials has not
// run): each block adds up those before it, and the last block writes the
// total (block 0 writes 0 when there is nothing to scan).
__global__ __launch_bounds__(B) void k_scan_down(ScanSrc src, uint32_t* out, int64_t max_count,
                                                 const uint32_t* dcount, const uint32_t* partial,
                                                 uint32_t* firsts, uint32_t firsts_len, bool direct,
                                                 uint32_t* total) {
  __shared__ uint32_t s_wave[kRounds][NW];
  __shared__ uint32_t s_pre[NW];
  const uint32_t n = dev_count(dcount, max_count);
  const uint64_t begin = (uint64_t)blockIdx.x * kSortChunk;
  if (begin >= n) {
    if (direct && total && blockIdx.x == 0 && threadIdx.x == 0) *total = 0u;
    return;
  }
  uint32_t v[kRounds][4];
  load_chunk(src, begin, n, v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  uint32_t s[kRounds], inc[kRounds];
#pragma unroll
  for (int r = 0; r < kRounds; ++r) {
    s[r] = (v[r][0] + v[r][1]) + (v[r][2] + v[r][3]);
    inc[r] = wave_incl_scan(s[r]);
    if (lane == 63) s_wave[r][w] = inc[r];
  }
  __syncthreads();
  uint32_t carry;
  if (direct) {
    uint32_t x = 0;
    for (uint32_t q = threadIdx.x; q < blockIdx.x; q += B) x += partial[q];
    block_excl_scan(x, s_pre, &carry);
  } else {
    carry = partial[blockIdx.x];
  }
  const bool full = begin + kSortChunk <= n && ((reinterpret_cast<uintptr_t>(out)) & 15u) == 0;
#pragma unroll
  for (int r = 0; r < kRounds; ++r) {
    uint32_t before = 0, tot = 0;
#pragma unroll
    for (int q = 0; q < NW; ++q) {
      const uint32_t x = s_wave[r][q];
      before += (q < w) ? x : 0u;
      tot += x;
    }
    uint32_t run = carry + before + inc[r] - s[r];
    carry += tot;
    const uint64_t k = begin + (uint64_t)r * 4 * B + 4u * threadIdx.x;
    uint32_t o[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      o[c] = run;
      run += v[r][c];
    }
    if (firsts) {
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        if (k + c >= n) continue;
        const uint64_t lo = o[c], hi = lo + v[r][c];
        for (uint64_t m = (lo + kSortChunk - 1) / kSortChunk; m < firsts_len && m * kSortChunk < hi; ++m)
          firsts[m] = (uint32_t)(k + c);
      }
    }
    if (full) {
      *reinterpret_cast<uint4*>(out + k) = make_uint4(o[0], o[1], o[2], o[3]);
    } else {
#pragma unroll
      for (int c = 0; c < 4; ++c)
        if (k + c < n) out[k + c] = o[c];
    }
  }
  if (direct && total && begin + kSortChunk >= n && threadIdx.x == 0) *total = carry;
}

__global__ void k_fill_u32(uint32_t* p, uint32_t value, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = value;
}

// ---- radix sort (LSD, digits of up to 8 bits, stable) -----------------------
// Digit counts of one chunk per workgroup; each thread loads its kSortItems
// keys with 16-byte loads (the scan chunk layout) and counts them with LDS
// atomics into one of kHistCopies interleaved copies of its wavefront's
// histogram (copy lane % kHistCopies; the copies of a digit are adjacent
// words, so in different banks).  A skewed digit (the exponent byte of depth
// keys) then meets at most 64 / kHistCopies lanes of one wavefront at each
// address instead of 64.  Counts are stored digit-major, hist[d * nblocks +
// chunk].
constexpr int kHistCopies = 4;

// With `valid` (the first depth pass, reading the dense (view, Gaussian)
// arrays), key k counts only where valid[k] != 0: the pass then compacts the
// visible pairs as it sorts them.
__global__ __launch_bounds__(B) void k_radix_hist(const uint32_t* keys, const uint32_t* valid, int64_t max_count,
                                                  const uint32_t* dcount, int shift, uint32_t dmask, int64_t nblocks,
                                                  uint32_t* hist) {
  __shared__ uint32_t h[NW][256][kHistCopies];
#pragma unroll
  for (int q = 0; q < NW * kHistCopies; ++q) (&h[0][0][0])[q * 256 + threadIdx.x] = 0;
  __syncthreads();
  const uint32_t n = dev_count(dcount, max_count);
  const int w = threadIdx.x >> 6, copy = threadIdx.x & (kHistCopies - 1);
  const int64_t chunk = blockIdx.x;
  const uint64_t begin = (uint64_t)chunk * kSortChunk;
  if (chunk < nblocks && begin < n) {
    uint32_t v[kRounds][4], ok[kRounds][4];
    load_chunk(ScanSrc{keys, nullptr, 0}, begin, n, v);
    if (valid) load_chunk(ScanSrc{valid, nullptr, 1}, begin, n, ok);
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
#pragma unroll
      for (int c = 0; c < 4; ++c)
        if (begin + (uint64_t)r * 4 * B + 4u * threadIdx.x + c < n && (!valid || ok[r][c]))
          atomicAdd(&h[w][(v[r][c] >> shift) & dmask][copy], 1u);
    }
  }
  __syncthreads();
  uint32_t t = 0;
#pragma unroll
  for (int q = 0; q < NW; ++q)
#pragma unroll
    for (int k = 0; k < kHistCopies; ++k) t += h[q][threadIdx.x][k];
  if (chunk < nblocks) hist[(int64_t)threadIdx.x * nblocks + chunk] = t;
}

// Scatter of one chunk (kSortChunk keys, split into NW contiguous wavefront
// ranges).  1) Each wavefront ranks its keys stably within (wavefront, digit):
// lanes with equal digits are matched with eight ballots and a per-wavefront
// counter per digit advances by the group size.  2) Per digit, the chunk-local
// start (scan over digits) and the start of each wavefront's group.  3) Keys
// are placed in LDS in digit order (stable), 4) then written out with
// consecutive threads taking consecutive local positions, so each digit's run
// is stored contiguously: global position = scanned histogram of (digit,
// chunk) + position within the digit's run.  With kPay, a 64-bit payload per
// key follows the same permutation through the same LDS space afterwards.
constexpr int kWaveKeys = kSortChunk / NW;
constexpr int kWaveRounds = kWaveKeys / 64;
constexpr int kOutRounds = kSortChunk / B;

// Steps 1-4 of a scatter for the keys a chunk's wavefronts hold (key[r] and
// val[r] of lane l of wavefront w are chunk entry w kWaveKeys + r 64 + l;
// bit r of in_mask says whether it takes part).  s_wc must be zero and
// visible to the whole workgroup on entry.  pos[] (each key's local
// position) and dst[] (with kPay: the global position of local entry
// r B + threadIdx.x) serve a payload that follows the keys; returns the
// number of keys taken.  With kBounded, positions at or past `limit` are not
// written (a safeguard where the digit counts come from another kernel's
// arithmetic rather than from the keys themselves).
template <bool kPay, bool kBounded = false>
__device__ __forceinline__ uint32_t rank_and_write(const uint32_t (&key)[kWaveRounds], const uint32_t (&val)[kWaveRounds],
                                                   uint32_t in_mask, uint32_t digit_base, int shift, uint32_t dmask,
                                                   uint32_t* s_key, uint32_t* s_val, uint32_t (*s_wc)[256],
                                                   uint32_t* s_gbase, uint32_t* s_tmp, uint32_t& s_taken,
                                                   uint32_t* kout, uint32_t* vout, uint32_t (&pos)[kWaveRounds],
                                                   uint32_t (&dst)[kPay ? kOutRounds : 1], uint32_t limit = 0u) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  uint32_t lr[kWaveRounds];
  // 1. stable ranks within (wavefront, digit)
#pragma unroll
  for (int r = 0; r < kWaveRounds; ++r) {
    const bool taking = (in_mask >> r) & 1u;
    const uint32_t digit = (key[r] >> shift) & dmask;
    uint64_t match = __ballot(taking);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (digit >> b) & 1u;
      const uint64_t bb = __ballot(bit);
      match &= bit ? bb : ~bb;
    }
    const uint32_t below = (uint32_t)__popcll(match & lt_mask);
    const uint32_t before = taking ? s_wc[w][digit] : 0u;
    __builtin_amdgcn_wave_barrier();
    lr[r] = before + below;
    if (taking && below == 0) s_wc[w][digit] = before + (uint32_t)__popcll(match);
    __builtin_amdgcn_wave_barrier();
  }
  __syncthreads();
  // 2. chunk-local digit starts and per-wavefront group starts
  {
    const int d = threadIdx.x;
    uint32_t c[NW], tot = 0;
#pragma unroll
    for (int q = 0; q < NW; ++q) {
      c[q] = s_wc[q][d];
      tot += c[q];
    }
    uint32_t all;
    const uint32_t lstart = block_excl_scan(tot, s_tmp, &all);
    if (d == 0) s_taken = all;
    uint32_t run = lstart;
#pragma unroll
    for (int q = 0; q < NW; ++q) {
      s_wc[q][d] = run;
      run += c[q];
    }
    s_gbase[d] = digit_base - lstart;
  }
  __syncthreads();
  // 3. local placement in digit order
#pragma unroll
  for (int r = 0; r < kWaveRounds; ++r) {
    pos[r] = s_wc[w][(key[r] >> shift) & dmask] + lr[r];
    if ((in_mask >> r) & 1u) {
      s_key[pos[r]] = key[r];
      s_val[pos[r]] = val[r];
    }
  }
  __syncthreads();
  // 4. coalesced write-out
  const uint32_t taken = s_taken;
#pragma unroll
  for (int r = 0; r < kOutRounds; ++r) {
    const uint32_t i = (uint32_t)r * B + threadIdx.x;
    if (i < taken) {
      const uint32_t k = s_key[i];
      const uint32_t d = s_gbase[(k >> shift) & dmask] + i;
      if (kBounded && d >= limit) continue;
      kout[d] = k;
      vout[d] = s_val[i];
      if constexpr (kPay) dst[r] = d;
    }
  }
  return taken;
}

// kDense (the first depth pass): the input is the dense (view, Gaussian)
// range, key k is taken only where valid[k] != 0, and its value is
// value_base + k (the pair's index), so the pass compacts the visible pairs
// in (view, Gaussian) order as it sorts them.
template <bool kPay, bool kDense = false>
__global__ __launch_bounds__(B) void k_radix_scatter(const uint32_t* kin, const uint32_t* vin, uint32_t* kout,
                                                     uint32_t* vout, const uint2* pin, uint2* pout,
                                                     int64_t max_count, const uint32_t* dcount, int shift,
                                                     uint32_t dmask, int64_t nblocks, const uint32_t* hist_scanned,
                                                     const uint32_t* valid = nullptr, uint32_t value_base = 0) {
  __shared__ __align__(16) uint32_t s_kv[2 * kSortChunk];   // keys | values, later the payload
  __shared__ uint32_t s_wc[NW][256];
  __shared__ uint32_t s_gbase[256];
  __shared__ uint32_t s_tmp[NW];
  __shared__ uint32_t s_taken;   // keys of the chunk that take part (all but invalid dense entries)
  uint32_t* s_key = s_kv;
  uint32_t* s_val = s_kv + kSortChunk;
  const uint32_t n = dev_count(dcount, max_count);
  const uint64_t begin = (uint64_t)blockIdx.x * kSortChunk;
  if (begin >= n) return;
  const uint32_t cnt = (uint32_t)min((uint64_t)kSortChunk, (uint64_t)n - begin);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < NW; ++q) s_wc[q][threadIdx.x] = 0;
  uint32_t key[kWaveRounds], val[kWaveRounds];
  uint2 pay[kPay ? kWaveRounds : 1];
  // Each pass reads its input once: streaming loads leave the cache to the
  // histogram, the offsets and the output being assembled.  Every load of
  // the chunk is issued before any result is used (a whole chunk, the common
  // case, loads without conditions; the validity flags of a dense pass are
  // turned into the taken mask only afterwards), and a dense pass loads every
  // entry's key and payload whether or not it takes it: taken and skipped
  // entries share cache lines.
  uint32_t flag[kDense ? kWaveRounds : 1];
  const uint32_t lane0 = (uint32_t)w * kWaveKeys + (uint32_t)lane;
  // this chunk's global start of digit threadIdx.x, needed only after the
  // ranking: loaded with the keys so that its latency overlaps theirs
  const uint32_t digit_base = hist_scanned[(int64_t)threadIdx.x * nblocks + blockIdx.x];
  if (cnt == (uint32_t)kSortChunk) {   // uniform
#pragma unroll
    for (int r = 0; r < kWaveRounds; ++r) {
      const uint64_t k = begin + lane0 + (uint32_t)r * 64u;
      key[r] = __builtin_nontemporal_load(kin + k);
      if constexpr (kDense)
        flag[r] = __builtin_nontemporal_load(valid + k);
      else
        val[r] = __builtin_nontemporal_load(vin + k);
      if constexpr (kPay) {
        const uint32_t* pp = reinterpret_cast<const uint32_t*>(pin + k);
        pay[r] = make_uint2(__builtin_nontemporal_load(pp), __builtin_nontemporal_load(pp + 1));
      }
    }
  } else {
#pragma unroll
    for (int r = 0; r < kWaveRounds; ++r) {
      const uint32_t li = lane0 + (uint32_t)r * 64u;
      const bool here = li < cnt;
      key[r] = here ? __builtin_nontemporal_load(kin + begin + li) : 0u;
      if constexpr (kDense)
        flag[r] = here ? __builtin_nontemporal_load(valid + begin + li) : 0u;
      else
        val[r] = here ? __builtin_nontemporal_load(vin + begin + li) : 0u;
      if constexpr (kPay) {
        if (here) {
          const uint32_t* pp = reinterpret_cast<const uint32_t*>(pin + begin + li);
          pay[r] = make_uint2(__builtin_nontemporal_load(pp), __builtin_nontemporal_load(pp + 1));
        } else {
          pay[r] = make_uint2(0u, 0u);
        }
      }
    }
  }
  uint32_t in_mask = 0;   // bit r: this lane's key of round r takes part
#pragma unroll
  for (int r = 0; r < kWaveRounds; ++r) {
    const uint32_t li = lane0 + (uint32_t)r * 64u;
    bool in = li < cnt;
    if constexpr (kDense) {
      in = in && flag[r] != 0u;
      val[r] = value_base + (uint32_t)(begin + li);
    }
    in_mask |= in ? 1u << r : 0u;
  }
  __syncthreads();
  uint32_t pos[kWaveRounds];
  uint32_t dst[kPay ? kOutRounds : 1];
  const uint32_t taken = rank_and_write<kPay>(key, val, in_mask, digit_base, shift, dmask, s_key, s_val, s_wc, s_gbase,
                                              s_tmp, s_taken, kout, vout, pos, dst);
  if constexpr (kPay) {
    uint2* s_pay = reinterpret_cast<uint2*>(s_kv);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kWaveRounds; ++r)
      if ((in_mask >> r) & 1u) s_pay[pos[r]] = pay[r];
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kOutRounds; ++r) {
      const uint32_t i = (uint32_t)r * B + threadIdx.x;
      if (i < taken) pout[dst[r]] = s_pay[i];
    }
  }
}

// ---- key emission in depth order -----------------------------------------
// Workgroup c produces the key slots [c K, (c+1) K) of one chunk of the tile
// sort (K = kSortChunk), twice: k_emit_count counts the digits of the sort's
// first pass over them, and after the scan of those counts k_emit_scatter
// produces them again and performs that first pass, so the keys in slot
// order are never stored.  Its wavefronts take the depth-sorted visible
// pairs from firsts[c], the pair owning slot c K, onwards, 64 consecutive
// pairs at a time, until a group starts past the chunk; a pair that
// straddles a chunk boundary is produced in part by both workgroups.  Within
// a group, lane l produces slot S + l in each round.  The pair owning a slot is found
// without searching: each pair whose first slot falls in the round marks that
// slot with its index, and an inclusive max-scan over the lanes (carried from
// the previous round, and started at the last pair that began at or before
// the chunk) hands every slot the last pair that started at or before it.
// The slot's tile within the pair's rectangle comes from a float-reciprocal
// quotient corrected to the exact integer one.

// Inclusive max-scan over the 64 lanes (values >= -1).
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ int dpp_max(int v) {
  return max(v, __builtin_amdgcn_update_dpp(-1, v, CTRL, ROW_MASK, 0xf, false));
}
__device__ __forceinline__ int wave_incl_max(int v) {
  v = dpp_max<0x111, 0xf>(v);   // row_shr:1
  v = dpp_max<0x112, 0xf>(v);   // row_shr:2
  v = dpp_max<0x114, 0xf>(v);   // row_shr:4
  v = dpp_max<0x118, 0xf>(v);   // row_shr:8
  v = dpp_max<0x142, 0xa>(v);   // row_bcast:15 into rows 1 and 3
  v = dpp_max<0x143, 0xc>(v);   // row_bcast:31 into rows 2 and 3
  return v;
}

// One lane's pair of a group of 64 depth-sorted visible pairs: first and
// end key slot, (view, Gaussian) index and tile rectangle as two words
// (x0 | y0 << 16, x1 | y1 << 16); past the last pair, off is 0xffffffff and
// the rest zero.
struct PairIn {
  uint32_t off, end, vi;
  uint2 r;
};

__device__ __forceinline__ PairIn load_pair(const uint32_t* koff, const uint32_t* sorted_vis, const uint2* sorted_rect,
                                            uint32_t k, uint32_t nvis, uint32_t all_keys) {
  PairIn p{0xffffffffu, 0u, 0u, make_uint2(0u, 0u)};
  if (k < nvis) {
    p.off = koff[k];
    p.end = k + 1 < nvis ? koff[k + 1] : all_keys;
    p.vi = sorted_vis[k];
    p.r = sorted_rect[k];
  }
  return p;
}

// Per-wavefront staging of the walk: the current group of 64 pairs.
struct WalkLds {
  uint32_t off[NW][64];    // first key slot
  uint32_t vi[NW][64];     // (view, Gaussian) index
  uint2 rect[NW][64];      // tile rectangle, as loaded
  uint32_t view[NW][64];
  int32_t mark[NW][64];
};

// The walk over chunk blockIdx.x of the key slots, [S0, S1): every slot is
// produced once, by one lane, which calls emit(slot, key, value).  s_view
// holds each view's (first tile relative to the call's first tile, tiles
// per row) and must be visible to the workgroup on entry.
template <class Emit>
__device__ __forceinline__ void emit_walk(WalkLds& L, const uint32_t* sorted_vis, const uint32_t* koff,
                                          const uint32_t* firsts, uint32_t nvis, uint32_t all_keys,
                                          const uint2* sorted_rect, const int2* s_view, uint32_t ng, uint64_t S0,
                                          uint32_t S1, Emit emit) {
  uint32_t (&s_off)[NW][64] = L.off;
  uint32_t (&s_vi)[NW][64] = L.vi;
  uint2 (&s_rect)[NW][64] = L.rect;
  uint32_t (&s_v)[NW][64] = L.view;
  int32_t (&s_mark)[NW][64] = L.mark;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const float inv_ng = 1.f / (float)ng;
  // the wavefront takes every NW-th group of 64 pairs; each group's loads go
  // out together, and before the group in hand is worked through, so that
  // they are in flight meanwhile
  uint32_t g = firsts[blockIdx.x] + (uint32_t)w * 64u;
  PairIn nxt = load_pair(koff, sorted_vis, sorted_rect, g + (uint32_t)lane, nvis, all_keys);
  for (; g < nvis; g += NW * 64u) {
    const PairIn cur = nxt;
    if ((uint32_t)__builtin_amdgcn_readfirstlane((int)cur.off) >= S1) break;   // the group starts past the chunk
    const bool valid = g + (uint32_t)lane < nvis;
    const uint32_t off = cur.off, vi = cur.vi;
    // view = vi / n_gauss: a float estimate (off by at most one, as the
    // quotient is below 2^8) corrected to the exact integer quotient (lanes
    // past the last pair stage zeros, which no slot refers to)
    uint32_t v = (uint32_t)((float)vi * inv_ng);
    const uint64_t lv = (uint64_t)v * ng;
    if (lv > vi) v -= 1u;
    else if (lv + ng <= vi) v += 1u;
    s_vi[w][lane] = vi;
    s_rect[w][lane] = cur.r;
    s_v[w][lane] = v;
    s_off[w][lane] = off;
    uint32_t stop = cur.end;
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) stop = max(stop, (uint32_t)__shfl_xor((int)stop, d, 64));
    stop = min(stop, S1);
    // every use of this group's loads is above, so the next group's loads
    // stay in flight while the group is worked through
    __builtin_amdgcn_sched_barrier(0);
    nxt = load_pair(koff, sorted_vis, sorted_rect, g + NW * 64u + (uint32_t)lane, nvis, all_keys);
    __builtin_amdgcn_wave_barrier();
    const uint32_t start = max(s_off[w][0], (uint32_t)S0);
    // the last pair of the group that began at or before `start`
    int carry = (int)__popcll(__ballot(valid && off <= start)) - 1;
    for (uint32_t S = start; S < stop; S += 64) {
      s_mark[w][lane] = -1;
      __builtin_amdgcn_wave_barrier();
      if (valid && off >= S && off - S < 64u) s_mark[w][off - S] = lane;
      __builtin_amdgcn_wave_barrier();
      const int own = wave_incl_max(max(s_mark[w][lane], carry));
      carry = __builtin_amdgcn_readlane(own, 63);
      __builtin_amdgcn_wave_barrier();
      const uint32_t slot = S + (uint32_t)lane;
      if (slot < stop) {
        const uint2 rr = s_rect[w][own];
        const uint32_t rx = rr.x & 0xffffu, ry = rr.x >> 16;
        const uint32_t m = slot - s_off[w][own];
        const uint32_t width = (rr.y & 0xffffu) - rx + 1u;
        uint32_t q = (uint32_t)((float)m * __builtin_amdgcn_rcpf((float)width));
        int32_t rem = (int32_t)(m - q * width);
        if (rem < 0) {
          q -= 1u;
          rem += (int32_t)width;
        } else if (rem >= (int32_t)width) {
          q += 1u;
          rem -= (int32_t)width;
        }
        const uint32_t ty = ry + q, tx = rx + (uint32_t)rem;
        const int2 vw = s_view[s_v[w][own]];
        const uint32_t key = (uint32_t)(vw.x + (int32_t)(ty * (uint32_t)vw.y + tx));
        emit(slot, key, s_vi[w][own]);
      }
    }
    __builtin_amdgcn_wave_barrier();
  }
}

// Digit counts of the tile sort's first pass (key bits dmask0, a power of
// two minus one) for every chunk, in the layout k_radix_hist writes
// (hist[d * nblocks + c]), without producing the keys: the keys a pair has
// in one tile row of its rectangle are consecutive integers, so the row adds
// one to every digit len / (dmask0 + 1) times and to a cyclic range of
// len % (dmask0 + 1) digits once.  Each lane takes one pair of the chunk
// (clipped to the chunk's slots) row by row; the ranges go into a
// difference array, whose prefix sums are the counts.
__global__ __launch_bounds__(B) void k_emit_count(const uint32_t* sorted_vis, const uint32_t* koff,
                                                  const uint32_t* firsts, const uint32_t* nvis_p,
                                                  const uint32_t* total_keys, const uint2* sorted_rect,
                                                  const ViewInfo* views, int32_t n_views, int64_t n_gauss,
                                                  int32_t tile_begin, uint32_t cap, int64_t nblocks, uint32_t dmask0,
                                                  uint32_t* hist) {
  __shared__ int32_t s_diff[257];
  __shared__ uint32_t s_full;
  __shared__ uint32_t s_tmp[NW];
  __shared__ int2 s_view[kMaxViews];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  s_diff[threadIdx.x] = 0;
  if (threadIdx.x == 0) {
    s_diff[256] = 0;
    s_full = 0u;
  }
  for (int v = threadIdx.x; v < n_views; v += B) s_view[v] = make_int2(views[v].tile_base - tile_begin, views[v].tiles_x);
  __syncthreads();
  const uint32_t all_keys = *total_keys;
  const uint32_t n = min(all_keys, cap);
  const uint32_t M = dmask0 + 1u;
  const int bits0 = __popc(dmask0);
  const uint64_t S0 = (uint64_t)blockIdx.x * kSortChunk;
  if (S0 < n) {
    const uint32_t S1 = (uint32_t)min((uint64_t)n, S0 + kSortChunk);
    const uint32_t nvis = *nvis_p;
    const uint32_t ng = (uint32_t)n_gauss;
    const float inv_ng = 1.f / (float)ng;
    // groups of 64 pairs as in the walk, the next group's loads issued
    // before the group in hand is counted
    uint32_t g = firsts[blockIdx.x] + (uint32_t)w * 64u;
    PairIn nxt = load_pair(koff, sorted_vis, sorted_rect, g + (uint32_t)lane, nvis, all_keys);
    for (; g < nvis; g += NW * 64u) {
      const PairIn cur = nxt;
      if ((uint32_t)__builtin_amdgcn_readfirstlane((int)cur.off) >= S1) break;   // the group starts past the chunk
      const bool valid = g + (uint32_t)lane < nvis;
      const uint32_t off = cur.off, vi = cur.vi;
      const uint32_t lo = max(off, (uint32_t)S0), hi = min(cur.end, S1);
      // everything taken from this group's loads, for every lane (lanes past
      // the last pair or outside the chunk compute values they never use)
      uint32_t v = (uint32_t)((float)vi * inv_ng);   // vi / n_gauss, corrected as in the walk
      const uint64_t lv = (uint64_t)v * ng;
      if (lv > vi) v -= 1u;
      else if (lv + ng <= vi) v += 1u;
      const int2 vw = s_view[v];
      // the rectangle's words pass through an empty asm statement here, so
      // that the compiler does not narrow the next group's rectangle load
      // right where it is issued (which would make the wavefront wait for it)
      uint32_t rw0 = cur.r.x, rw1 = cur.r.y;
      asm volatile("" : "+v"(rw0), "+v"(rw1));
      const uint32_t rx = rw0 & 0xffffu, ry = rw0 >> 16;
      const uint32_t width = (rw1 & 0xffffu) - rx + 1u;
      const uint32_t m0 = lo - off, m1 = hi - off;   // the pair's slots in the chunk, [m0, m1)
      const uint32_t q0 = m0 / width, c0 = m0 - q0 * width;
      const uint32_t q1 = (m1 - 1u) / width, c1 = (m1 - 1u) - q1 * width;
      // so the next group's loads stay in flight while this one is counted
      __builtin_amdgcn_sched_barrier(0);
      nxt = load_pair(koff, sorted_vis, sorted_rect, g + NW * 64u + (uint32_t)lane, nvis, all_keys);
      if (valid && lo < hi) {
        uint32_t full = 0;
        for (uint32_t q = q0; q <= q1; ++q) {
          const uint32_t cs = q == q0 ? c0 : 0u, ce = q == q1 ? c1 : width - 1u;
          const uint32_t a = (uint32_t)(vw.x + (int32_t)((ry + q) * (uint32_t)vw.y + rx + cs));
          const uint32_t len = ce - cs + 1u;
          full += len >> bits0;
          const uint32_t rem = len & dmask0;
          if (rem) {
            const uint32_t s = a & dmask0, e = s + rem;
            atomicAdd(&s_diff[s], 1);
            if (e < M) {
              atomicAdd(&s_diff[e], -1);
            } else if (e > M) {
              atomicAdd(&s_diff[0], 1);
              atomicAdd(&s_diff[e - M], -1);
            }
          }
        }
        if (full) atomicAdd(&s_full, full);
      }
    }
  }
  __syncthreads();
  const uint32_t d = threadIdx.x;
  const int32_t x = d < M ? s_diff[d] : 0;
  uint32_t total;
  const uint32_t below = block_excl_scan((uint32_t)x, s_tmp, &total);
  hist[(int64_t)d * nblocks + blockIdx.x] = d < M ? below + (uint32_t)x + s_full : 0u;
}

// The tile sort's first pass fused with the key emission: workgroup c walks
// its chunk's slots again, places each (key, value) at its slot in LDS, and
// then ranks and scatters them as k_radix_scatter does (digits key & dmask0,
// hist_scanned the scanned counts of k_emit_count), so the emitted keys
// never go through HBM in slot order.  Its LDS use is kept at 40 KB (the
// walk's staging shares space with the ranking's counters) for four
// workgroups per compute unit; with 48 KB and three it was no faster than
// emitting and sorting in separate kernels.
__global__ __launch_bounds__(B) void k_emit_scatter(const uint32_t* sorted_vis, const uint32_t* koff,
                                                    const uint32_t* firsts, const uint32_t* nvis_p,
                                                    const uint32_t* total_keys, const uint2* sorted_rect,
                                                    const ViewInfo* views, int32_t n_views, int64_t n_gauss,
                                                    int32_t tile_begin, uint32_t cap, int64_t nblocks, uint32_t dmask0,
                                                    const uint32_t* hist_scanned, uint32_t* kout, uint32_t* vout) {
  __shared__ __align__(16) uint32_t s_kv[2 * kSortChunk];   // keys | values
  __shared__ int2 s_view[kMaxViews];
  __shared__ union {   // the walk's staging, then the ranking's counters
    WalkLds walk;
    struct {
      uint32_t wc[NW][256];
      uint32_t gbase[256];
      uint32_t tmp[NW];
      uint32_t taken;
    } rank;
  } u;
  uint32_t* s_key = s_kv;
  uint32_t* s_val = s_kv + kSortChunk;
  const uint32_t all_keys = *total_keys;
  const uint32_t n = min(all_keys, cap);
  const uint64_t S0 = (uint64_t)blockIdx.x * kSortChunk;
  if (S0 >= n) return;
  const uint32_t S1 = (uint32_t)min((uint64_t)n, S0 + kSortChunk);
  const uint32_t cnt = S1 - (uint32_t)S0;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int v = threadIdx.x; v < n_views; v += B) s_view[v] = make_int2(views[v].tile_base - tile_begin, views[v].tiles_x);
  const uint32_t digit_base = hist_scanned[(int64_t)threadIdx.x * nblocks + blockIdx.x];
  __syncthreads();
  emit_walk(u.walk, sorted_vis, koff, firsts, *nvis_p, all_keys, sorted_rect, s_view, (uint32_t)n_gauss, S0, S1,
            [&](uint32_t slot, uint32_t key, uint32_t val) {
              s_key[slot - (uint32_t)S0] = key;
              s_val[slot - (uint32_t)S0] = val;
            });
  __syncthreads();
  uint32_t key[kWaveRounds], val[kWaveRounds];
  uint32_t in_mask = 0;
  const uint32_t lane0 = (uint32_t)w * kWaveKeys + (uint32_t)lane;
#pragma unroll
  for (int r = 0; r < kWaveRounds; ++r) {
    const uint32_t li = lane0 + (uint32_t)r * 64u;
    const bool in = li < cnt;
    key[r] = in ? s_key[li] : 0u;
    val[r] = in ? s_val[li] : 0u;
    in_mask |= in ? 1u << r : 0u;
  }
#pragma unroll
  for (int q = 0; q < NW; ++q) u.rank.wc[q][threadIdx.x] = 0;
  // the ranking places keys into the same LDS space
  __syncthreads();
  uint32_t pos[kWaveRounds];
  uint32_t dst[1];
  rank_and_write<false, true>(key, val, in_mask, digit_base, 0, dmask0, s_key, s_val, u.rank.wc, u.rank.gbase,
                              u.rank.tmp, u.rank.taken, kout, vout, pos, dst, n);
}

__global__ void k_key_total(Counters* c, const uint32_t* total_keys, uint32_t cap) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    const uint32_t k = *total_keys;
    c->keys = k;
    c->key_cap = cap;
    if (k > cap) {
      c->overflow = 1u;
      c->overflow_any = 1u;
    }
  }
}

// Per-tile [start, end) of the sorted keys; thread q looks at keys 4q..4q+3
// (one 16-byte load) and their two outer neighbours.
__global__ __launch_bounds__(256) void k_ranges(const uint32_t* keys, const uint32_t* count_p, uint32_t cap,
                                                int32_t tile_begin, uint2* ranges) {
  constexpr uint32_t kNone = 0xffffffffu;   // no tile id reaches this
  const uint32_t n = min(*count_p, cap);
  const uint32_t nq = (n + 3u) / 4u;
  const bool aligned = (reinterpret_cast<uintptr_t>(keys) & 15u) == 0;
  const uint32_t lane = threadIdx.x & 63u;
  // whole wavefronts go round the loop together (lanes past the last quad
  // hold kNone), so that each quad's outer neighbours, the last key of the
  // quad before and the first of the quad after, come from the lanes beside
  // it
  for (uint32_t qb = blockIdx.x * blockDim.x + (threadIdx.x & ~63u); qb < nq; qb += gridDim.x * blockDim.x) {
    const uint32_t qd = qb + lane;
    const bool here = qd < nq;
    const uint32_t k0 = qd * 4u;
    uint32_t t[6];
    if (here && aligned && k0 + 4u <= n) {
      typedef uint32_t U4 __attribute__((ext_vector_type(4)));
      const U4 x = __builtin_nontemporal_load(reinterpret_cast<const U4*>(keys + k0));
      t[1] = x.x, t[2] = x.y, t[3] = x.z, t[4] = x.w;
    } else {
#pragma unroll
      for (int c = 0; c < 4; ++c) t[1 + c] = here && k0 + c < n ? keys[k0 + c] : kNone;
    }
    // lane 0's key before its quad and lane 63's key after it, in flight
    // together with the quads
    uint32_t before = kNone, after = kNone;
    if (lane == 0u && here && k0 > 0u) before = keys[k0 - 1u];
    if (lane == 63u && here && k0 + 4u < n) after = keys[k0 + 4u];
    t[0] = (uint32_t)__shfl_up((int)t[4], 1, 64);
    t[5] = (uint32_t)__shfl_down((int)t[1], 1, 64);
    if (lane == 0u) t[0] = before;
    if (lane == 63u) t[5] = after;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const uint32_t k = k0 + c;
      if (here && k < n) {
        if (t[c] != t[c + 1]) ranges[tile_begin + t[c + 1]].x = k;
        if (t[c + 2] != t[c + 1]) ranges[tile_begin + t[c + 1]].y = k + 1u;
      }
    }
  }
}

// ---- longest-first tile order (persistent compositing, schedule 3) ----------
// Tiles are bucketed by the bit length of their list length (0 for an empty
// list), longer buckets first; within a bucket a workgroup's tiles keep
// their row-major neighbourhood.  Only the order in which tiles are handed
// out depends on it, never a result.
constexpr int kOrderBuckets = 33;

__device__ __forceinline__ uint32_t list_bucket(uint2 r) {
  const uint32_t n = r.y > r.x ? r.y - r.x : 0u;
  return 32u - (uint32_t)__clz(n);
}

__global__ __launch_bounds__(256) void k_order_hist(const uint2* ranges, uint32_t ntiles, uint32_t* bkt) {
  __shared__ uint32_t h[kOrderBuckets];
  if (threadIdx.x < kOrderBuckets) h[threadIdx.x] = 0u;
  __syncthreads();
  const uint32_t t = blockIdx.x * 256u + threadIdx.x;
  if (t < ntiles) atomicAdd(&h[list_bucket(ranges[t])], 1u);
  __syncthreads();
  if (threadIdx.x < kOrderBuckets && h[threadIdx.x] != 0u) atomicAdd(&bkt[threadIdx.x], h[threadIdx.x]);
}

// bkt[0..32]: tiles per bucket (complete); bkt[33..65]: cursors, zero at start
__global__ __launch_bounds__(256) void k_order_scatter(const uint2* ranges, uint32_t ntiles, uint32_t* bkt,
                                                       uint32_t* order) {
  __shared__ uint32_t h[kOrderBuckets];
  __shared__ uint32_t base[kOrderBuckets];
  if (threadIdx.x < kOrderBuckets) h[threadIdx.x] = 0u;
  __syncthreads();
  const uint32_t t = blockIdx.x * 256u + threadIdx.x;
  uint32_t b = 0, r = 0;
  if (t < ntiles) {
    b = list_bucket(ranges[t]);
    r = atomicAdd(&h[b], 1u);
  }
  __syncthreads();
  if (threadIdx.x < kOrderBuckets && h[threadIdx.x] != 0u) {
    const uint32_t me = threadIdx.x;
    uint32_t start = 0;
    for (uint32_t q = me + 1; q < (uint32_t)kOrderBuckets; ++q) start += bkt[q];
    base[me] = start + atomicAdd(&bkt[kOrderBuckets + me], h[me]);
  }
  __syncthreads();
  if (t < ntiles) order[base[b] + r] = t;
}

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace

hipError_t launch_fill_u32(uint32_t* p, uint32_t value, int64_t count, hipStream_t st) {
  if (count > 0) hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)cdiv(count, 256)), dim3(256), 0, st, p, value, count);
  return hipGetLastError();
}

static hipError_t scan_src(ScanSrc src, uint32_t* out, int64_t max_count, const uint32_t* dcount, uint32_t* partial,
                           int64_t partial_len, uint32_t* total, hipStream_t st, uint32_t* firsts = nullptr,
                           uint32_t firsts_len = 0) {
  const int64_t nb = cdiv(max_count, kSortChunk);
  if (nb + 1 > partial_len) return hipErrorInvalidValue;
  // up to kDirectScanBlocks chunks, each down-sweep block adds up the chunk
  // sums before it itself (at most that many reads per block) instead of a
  // single-workgroup scan of them in a launch of its own
  constexpr int64_t kDirectScanBlocks = 4096;
  const bool direct = nb > 0 && nb <= kDirectScanBlocks;
  if (nb > 0) {
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(B), 0, st, src, max_count, dcount, partial);
  }
  if (!direct) hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(1024), 0, st, max_count, dcount, partial, total);
  if (nb > 0) {
    hipLaunchKernelGGL(k_scan_down, dim3((unsigned)nb), dim3(B), 0, st, src, out, max_count, dcount, partial, firsts,
                       firsts_len, direct, total);
  }
  return hipGetLastError();
}

hipError_t launch_scan(const uint32_t* in, uint32_t* out, int64_t max_count, const uint32_t* dcount, uint32_t* partial,
                       int64_t partial_len, uint32_t* total, hipStream_t st) {
  return scan_src(ScanSrc{in, nullptr, 0}, out, max_count, dcount, partial, partial_len, total, st);
}

// Dense source of a sort's first pass: max_count keys key[k] with payload
// pay[k], taken only where valid[k] != 0, with value value_base + k; the
// number taken is written to *taken, which the later passes read as their
// count.
struct DenseSrc {
  const uint32_t* key;
  const uint32_t* valid;
  const uint2* pay;
  uint32_t value_base;
  uint32_t* taken;
};

// Sorts (key, value) pairs on key bits [0, bits) in ping-pong buffers, the
// first pass on the low first_bits bits and every later one on the next 8;
// returns through *in_b whether the result landed in the second buffer.  With `dense`,
// the first pass reads the dense source instead of (ka, va, pa) and writes
// the taken keys to (ka, va, pa), and the later passes sort *dense->taken of
// them (dcount must then be dense->taken).  With first_done, the caller has
// already performed the first pass into (kb, vb, pb).
static hipError_t radix_sort(const Plan& pl, void* ws, uint32_t* ka, uint32_t* va, uint32_t* kb, uint32_t* vb,
                             uint2* pa, uint2* pb, int64_t max_count, const uint32_t* dcount, int bits, bool* in_b,
                             hipStream_t st, const DenseSrc* dense = nullptr, bool first_done = false,
                             int first_bits = 8) {
  const int64_t nb = cdiv(max_count, kSortChunk);
  uint32_t* hist = seg<uint32_t>(ws, pl.ws.hist);
  uint32_t* partial = seg<uint32_t>(ws, pl.ws.partial);
  if (nb > pl.ws.hist_blocks) return hipErrorInvalidValue;
  if (dense && (!pa || dcount != dense->taken)) return hipErrorInvalidValue;
  bool cur_b = false;   // which buffer holds the data (before a dense first pass: neither)
  for (int shift = 0; shift < bits; shift += (shift == 0 ? first_bits : 8)) {
    const uint32_t dmask = (1u << (shift == 0 ? first_bits : 8)) - 1u;
    const bool from_dense = dense && shift == 0;
    const bool out_b = from_dense ? false : !cur_b;
    const uint32_t* ki = from_dense ? dense->key : cur_b ? kb : ka;
    const uint32_t* vi = from_dense ? nullptr : cur_b ? vb : va;
    const uint2* pi = from_dense ? dense->pay : cur_b ? pb : pa;
    uint32_t* ko = out_b ? kb : ka;
    uint32_t* vo = out_b ? vb : va;
    uint2* po = out_b ? pb : pa;
    if (first_done && shift == 0) {
      cur_b = true;
      continue;
    }
    if (nb > 0) {
      const uint32_t* dc = from_dense ? nullptr : dcount;
      hipLaunchKernelGGL(k_radix_hist, dim3((unsigned)nb), dim3(B), 0, st, ki, from_dense ? dense->valid : nullptr,
                         max_count, dc, shift, dmask, nb, hist);
      // a dense pass's digit counts total the taken keys
      hipError_t e = scan_src(ScanSrc{hist, nullptr, 0}, hist, 256 * nb, nullptr, partial, pl.ws.partial_len,
                              from_dense ? dense->taken : nullptr, st);
      if (e != hipSuccess) return e;
      if (from_dense)
        hipLaunchKernelGGL((k_radix_scatter<true, true>), dim3((unsigned)nb), dim3(B), 0, st, ki, vi, ko, vo, pi, po,
                           max_count, dc, shift, dmask, nb, hist, dense->valid, dense->value_base);
      else if (pa)
        hipLaunchKernelGGL((k_radix_scatter<true, false>), dim3((unsigned)nb), dim3(B), 0, st, ki, vi, ko, vo, pi,
                           po, max_count, dc, shift, dmask, nb, hist, nullptr, 0u);
      else
        hipLaunchKernelGGL((k_radix_scatter<false, false>), dim3((unsigned)nb), dim3(B), 0, st, ki, vi, ko, vo, pi,
                           po, max_count, dc, shift, dmask, nb, hist, nullptr, 0u);
    } else if (from_dense) {
      hipError_t e = launch_fill_u32(dense->taken, 0u, 1, st);
      if (e != hipSuccess) return e;
    }
    cur_b = out_b;
  }
  *in_b = cur_b;
  return hipGetLastError();
}

hipError_t launch_sort_pairs(const Plan& pl, void* ws, uint32_t* ka, uint32_t* va, uint32_t* kb, uint32_t* vb,
                             int64_t count, int bits, bool* in_b, hipStream_t st) {
  return radix_sort(pl, ws, ka, va, kb, vb, nullptr, nullptr, count, nullptr, bits, in_b, st);
}

hipError_t launch_tile_lists(const Plan& pl, int v0, int nv, void* ws, hipStream_t st) {
  Counters* ctr = seg<Counters>(ws, pl.ws.counters);
  const int64_t N = pl.n;
  const int64_t base = (int64_t)v0 * N, len = (int64_t)nv * N;
  uint32_t* count = seg<uint32_t>(ws, pl.ws.count);
  uint32_t* depth = seg<uint32_t>(ws, pl.ws.depth);
  uint32_t* vis_a = seg<uint32_t>(ws, pl.ws.vis_a);
  uint32_t* vis_b = seg<uint32_t>(ws, pl.ws.vis_b);
  uint32_t* vkey_a = seg<uint32_t>(ws, pl.ws.vkey_a);
  uint32_t* vkey_b = seg<uint32_t>(ws, pl.ws.vkey_b);
  uint32_t* koff = seg<uint32_t>(ws, pl.ws.koff);
  uint2* vrect_a = seg<uint2>(ws, pl.ws.vrect_a);
  uint2* vrect_b = seg<uint2>(ws, pl.ws.vrect_b);
  uint32_t* partial = seg<uint32_t>(ws, pl.ws.partial);
  uint32_t* keys_a = seg<uint32_t>(ws, pl.ws.keys_a);
  uint32_t* keys_b = seg<uint32_t>(ws, pl.ws.keys_b);
  uint32_t* vals_a = seg<uint32_t>(ws, pl.ws.vals_a);
  uint32_t* vals_b = seg<uint32_t>(ws, pl.ws.vals_b);
  uint2* ranges = seg<uint2>(ws, pl.ws.ranges);
  const uint32_t cap = (uint32_t)pl.cap;
  hipError_t e;
  if (len == 0) return hipSuccess;
  // 1-2. stable depth sort of the visible pairs (ties keep (view, Gaussian)
  // order); its first pass reads the dense (view, Gaussian) arrays and takes
  // the visible pairs only, so it also compacts them and counts them into
  // ctr->nvis
  bool in_b = false;
  const DenseSrc dense{depth + base, count + base, seg<uint2>(ws, pl.ws.rect) + base, (uint32_t)base, &ctr->nvis};
  e = radix_sort(pl, ws, vkey_a, vis_a, vkey_b, vis_b, vrect_a, vrect_b, len, &ctr->nvis, 32, &in_b, st, &dense);
  if (e != hipSuccess) return e;
  const uint32_t* sorted_vis = in_b ? vis_b : vis_a;
  const uint2* sorted_rect = in_b ? vrect_b : vrect_a;
  // 3. key offsets in depth order, and the pair owning the first slot of
  // each chunk of the tile sort
  const int64_t key_chunks = cdiv(pl.cap, kSortChunk);
  if (key_chunks > pl.ws.hist_blocks) return hipErrorInvalidValue;
  uint32_t* firsts = seg<uint32_t>(ws, pl.ws.firsts);
  e = scan_src(ScanSrc{reinterpret_cast<const uint32_t*>(sorted_rect), nullptr, 3}, koff, len, &ctr->nvis, partial,
               pl.ws.partial_len, &ctr->keys, st, firsts, (uint32_t)key_chunks);
  if (e != hipSuccess) return e;
  // ctr->keys holds the total; record it and the overflow flag
  hipLaunchKernelGGL(k_key_total, dim3(1), dim3(64), 0, st, ctr, &ctr->keys, cap);
  // 4. digit counts of the tile sort's first pass over the (tile, value)
  // pairs in depth order, one sort chunk per workgroup, and their scan
  const int32_t tile_begin = pl.views[v0].tile_base;
  const int32_t tile_end = (v0 + nv < pl.n_views) ? pl.views[v0 + nv].tile_base : pl.total_tiles;
  // tile bits of the call, split into passes of 8 bits with the remainder
  // taken first: fewer digits in the first pass
  const int64_t ntiles = tile_end - tile_begin;
  int bits = 0;
  while ((1ll << bits) < ntiles) ++bits;
  if (bits == 0) bits = 1;
  const int first_bits = bits - 8 * ((bits - 1) / 8);
  uint32_t* hist = seg<uint32_t>(ws, pl.ws.hist);
  const uint32_t dmask0 = (1u << first_bits) - 1u;
  hipLaunchKernelGGL(k_emit_count, dim3((unsigned)key_chunks), dim3(B), 0, st, sorted_vis, koff, firsts, &ctr->nvis,
                     &ctr->keys, sorted_rect, pl.d_views, pl.n_views, N, tile_begin, cap, key_chunks, dmask0, hist);
  e = scan_src(ScanSrc{hist, nullptr, 0}, hist, 256 * key_chunks, nullptr, partial, pl.ws.partial_len, nullptr, st);
  if (e != hipSuccess) return e;
  // 5. stable sort by tile (relative to the first tile of the call): its
  // first pass fused with the emission, into the second buffers
  hipLaunchKernelGGL(k_emit_scatter, dim3((unsigned)key_chunks), dim3(B), 0, st, sorted_vis, koff, firsts, &ctr->nvis,
                     &ctr->keys, sorted_rect, pl.d_views, pl.n_views, N, tile_begin, cap, key_chunks, dmask0, hist, keys_b,
                     vals_b);
  e = radix_sort(pl, ws, keys_a, vals_a, keys_b, vals_b, nullptr, nullptr, pl.cap, &ctr->keys, bits, &in_b, st, nullptr,
                 true, first_bits);
  if (e != hipSuccess) return e;
  // 6. ranges
  e = launch_fill_u32(reinterpret_cast<uint32_t*>(ranges + tile_begin), 0u, 2 * ntiles, st);
  if (e != hipSuccess) return e;
  const uint32_t* sk = in_b ? keys_b : keys_a;
  // one quad of keys per thread (the loop in the kernel covers any size):
  // every wavefront's loads are in flight at once instead of one quad after
  // another per thread
  const int64_t rblocks = cdiv(cdiv(pl.cap, 4), 256) < 0x7fffffffll ? cdiv(cdiv(pl.cap, 4), 256) : 0x7fffffffll;
  hipLaunchKernelGGL(k_ranges, dim3((unsigned)rblocks), dim3(256), 0, st, sk, &ctr->keys, cap, tile_begin, ranges);
  // 7. longest-first order of the call's tiles for the persistent compositing kernels
  if (pl.schedule == 3 && ntiles > 0) {
    uint32_t* bkt = seg<uint32_t>(ws, pl.ws.obucket);
    e = launch_fill_u32(bkt, 0u, 2 * kOrderBuckets, st);
    if (e != hipSuccess) return e;
    const unsigned ob = (unsigned)cdiv(ntiles, 256);
    hipLaunchKernelGGL(k_order_hist, dim3(ob), dim3(256), 0, st, ranges + tile_begin, (uint32_t)ntiles, bkt);
    hipLaunchKernelGGL(k_order_scatter, dim3(ob), dim3(256), 0, st, ranges + tile_begin, (uint32_t)ntiles, bkt,
                       seg<uint32_t>(ws, pl.ws.order));
  }
  return hipGetLastError();
}

}  // namespace gs
