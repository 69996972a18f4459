// Device helpers shared by the filter kernels: cross-block memory accesses,
// the grid barrier, team (one island) and block reductions, the island
// pair-mean and pair-selection probability.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dev_math.h"

namespace airpf {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;


__device__ __forceinline__ int64_t tree_off(int m, int level) {  // level >= 1
  return 2 * static_cast<int64_t>(m) - ((2 * static_cast<int64_t>(m)) >> (level - 1));
}

__device__ __forceinline__ double ninf() { return -__longlong_as_double(0x7ff0000000000000LL); }

// log((exp(a) + exp(b)) / 2), symmetric in (a, b)
__device__ __forceinline__ double pair_mean(double a, double b) {
  const double hi = a > b ? a : b, lo = a > b ? b : a;
  if (hi == ninf()) return hi;
  double t = dexp(lo - hi);
  t = 1.0 + t;
  t = dlog(t);
  return (hi + t) - kLn2;
}

// log(exp(a) + exp(b)), symmetric in (a, b)
__device__ __forceinline__ double log_add_exp(double a, double b) {
  const double hi = a > b ? a : b, lo = a > b ? b : a;
  if (hi == ninf()) return hi;
  double t = dexp(lo - hi);
  t = 1.0 + t;
  t = dlog(t);
  return hi + t;
}

// probability that an island with log-weight lk takes its partner's block
__device__ __forceinline__ double take_partner_prob(double lk, double lp) {
  if (lp == ninf()) return 0.0;
  if (lk == ninf()) return 1.0;
  return 1.0 / (1.0 + dexp(lk - lp));
}

// ------------------------------------------------------------ cross-block data
// Everything one block writes for another (resampled blocks, the island tree,
// the ENF partials, barrier flags) is written and read with device-scope
// relaxed atomic accesses, which are coherent across the chip's per-XCD L2
// caches by themselves.  No device-scope fence is ever issued: on this part
// such a fence writes back or invalidates a whole L2, and an invalidated L2
// costs every block its cached code and arguments.
template <typename T>
__device__ __forceinline__ void put(T* p, T v) { __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }
template <typename T>
__device__ __forceinline__ T get(const T* p) {
  return __hip_atomic_load(const_cast<T*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ------------------------------------------------------------ grid barrier
// Flag-array barrier: block b publishes the epoch it has reached in flags[b]
// (its own word, so no two blocks ever update one address), and every block
// polls all G flags, lane t watching flags t, t + 256, ...  Before a block
// publishes, every lane waits until all of its memory operations have
// completed (s_waitcnt 0), so the block's device-scope stores are visible
// to any device-scope load issued after the flag is seen.  Spinning is
// bounded: after ~2^24 polls a block raises status and leaves.
__device__ bool grid_barrier(unsigned* flags, int G, int bid, unsigned& epoch, int* status) {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  ++epoch;
  if (threadIdx.x == 0) put(&flags[bid], epoch);
  int ok = 1;
  for (int i = threadIdx.x; i < G && ok; i += kBlock) {
    unsigned spins = 0;
    while (get(&flags[i]) < epoch) {
      __builtin_amdgcn_s_sleep(1);
      if ((++spins & 1023u) == 0 && (spins > (1u << 24) || get(status) != 0)) {
        put(status, 1);
        ok = 0;
        break;
      }
    }
  }
  ok = __syncthreads_and(ok);
  return ok != 0;
}

// ------------------------------------------------------------ team / block reductions
// A team is TP consecutive lanes (TP a power of two); TP <= 64 stays inside
// one wave (shuffles only), TP > 64 spans TP/64 whole waves (LDS combine).
// Every helper is called by the whole block (TP is block-uniform).

// Orders the LDS accesses of a team.  A team of TP <= 64 lanes lies inside
// one wave, whose LDS instructions execute in program order, so only the
// compiler has to be kept from moving accesses across this point; a wider
// team needs the block barrier.
__device__ __forceinline__ void team_sync(int TP) {
  if (TP <= 64) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

template <typename T>
__device__ __forceinline__ T team_bcast(T v, int TP, T* lds_slot_per_team) {
  const int tid = threadIdx.x;
  if (TP <= 64) return __shfl(v, (tid & 63) & ~(TP - 1), 64);
  const int team = tid / TP;
  if ((tid & (TP - 1)) == 0) lds_slot_per_team[team] = v;
  __syncthreads();
  const T r = lds_slot_per_team[team];
  __syncthreads();
  return r;
}

__device__ __forceinline__ double team_max(double v, int TP, double* red) {
  const int w = TP < 64 ? TP : 64;
  for (int d = 1; d < w; d <<= 1) v = fmax(v, __shfl_xor(v, d, 64));
  if (TP > 64) {
    const int tid = threadIdx.x;
    if ((tid & 63) == 0) red[tid >> 6] = v;
    __syncthreads();
    const int w0 = (tid / TP) * (TP >> 6);
    double r = red[w0];
    for (int i = 1; i < (TP >> 6); ++i) r = fmax(r, red[w0 + i]);
    __syncthreads();
    v = r;
  }
  return v;
}

__device__ __forceinline__ uint64_t team_sum_u64(uint64_t v, int TP, uint64_t* red) {
  const int w = TP < 64 ? TP : 64;
  for (int d = 1; d < w; d <<= 1) v += __shfl_xor(v, d, 64);
  if (TP > 64) {
    const int tid = threadIdx.x;
    if ((tid & 63) == 0) red[tid >> 6] = v;
    __syncthreads();
    const int w0 = (tid / TP) * (TP >> 6);
    uint64_t r = 0;
    for (int i = 0; i < (TP >> 6); ++i) r += red[w0 + i];
    __syncthreads();
    v = r;
  }
  return v;
}

// inclusive scan of v over the team's lanes (lane order)
__device__ __forceinline__ uint64_t team_scan_u64(uint64_t v, int TP, uint64_t* red) {
  const int tid = threadIdx.x;
  const int w = TP < 64 ? TP : 64;
  const int sl = tid & (w - 1);
  for (int d = 1; d < w; d <<= 1) {
    const uint64_t t = __shfl_up(v, d, w);
    if (sl >= d) v += t;
  }
  if (TP > 64) {
    if ((tid & 63) == 63) red[tid >> 6] = v;
    __syncthreads();
    const int w0 = (tid / TP) * (TP >> 6);
    uint64_t add = 0;
    for (int i = w0; i < (tid >> 6); ++i) add += red[i];
    __syncthreads();
    v += add;
  }
  return v;
}

// sum of a double over the team's lanes (fixed pattern; every lane gets it)
__device__ __forceinline__ double team_sum_f64(double v, int TP, double* red) {
  const int w = TP < 64 ? TP : 64;
  for (int d = 1; d < w; d <<= 1) v += __shfl_xor(v, d, 64);
  if (TP > 64) {
    const int tid = threadIdx.x;
    if ((tid & 63) == 0) red[tid >> 6] = v;
    __syncthreads();
    const int w0 = (tid / TP) * (TP >> 6);
    double r = 0.0;
    for (int i = 0; i < (TP >> 6); ++i) r += red[w0 + i];
    __syncthreads();
    v = r;
  }
  return v;
}

// inclusive scan of a double over the team's lanes (lane order)
__device__ __forceinline__ double team_scan_f64(double v, int TP, double* red) {
  const int tid = threadIdx.x;
  const int w = TP < 64 ? TP : 64;
  const int sl = tid & (w - 1);
  for (int d = 1; d < w; d <<= 1) {
    const double t = __shfl_up(v, d, w);
    if (sl >= d) v += t;
  }
  if (TP > 64) {
    if ((tid & 63) == 63) red[tid >> 6] = v;
    __syncthreads();
    const int w0 = (tid / TP) * (TP >> 6);
    double add = 0.0;
    for (int i = w0; i < (tid >> 6); ++i) add += red[i];
    __syncthreads();
    v += add;
  }
  return v;
}

// ENF sums of a set of island log-weights L: the record (M, a, b) holds
// M = max L, a = sum exp(L - M), b = sum exp(L - M)^2.  Records of two
// halves combine by rescaling to the larger maximum; a member at the maximum
// contributes exactly 1, as in the definition ENF = (m^-1 sum W)^2 / (m^-1 sum W^2)
// evaluated with W = exp(L - max L).
struct EnfRec { double M, a, b; };

__device__ __forceinline__ EnfRec enf_leaf(double L) {
  return L == ninf() ? EnfRec{L, 0.0, 0.0} : EnfRec{L, 1.0, 1.0};
}

// (the side at the larger maximum keeps its sums unscaled: its factor is
// exp(0) = 1 exactly, so one exponential per join suffices)
__device__ __forceinline__ EnfRec enf_join(const EnfRec& x, const EnfRec& y) {
  if (x.M == ninf()) return y;
  if (y.M == ninf()) return x;
  if (x.M >= y.M) {
    const double f = dexp(y.M - x.M);
    return EnfRec{x.M, x.a + y.a * f, x.b + y.b * (f * f)};
  }
  const double f = dexp(x.M - y.M);
  return EnfRec{y.M, x.a * f + y.a, x.b * (f * f) + y.b};
}

// reduce n = 2^q records in LDS (arrays M, A, B) by adjacent pairs, whole
// block; w* are scratch arrays of n/2.  The pairing depends only on the
// indices, so records of aligned index ranges combine to the same value
// however the range is split across blocks.
__device__ EnfRec block_pair_enf(double* M, double* A, double* B, double* wM, double* wA, double* wB, int n) {
  double *sm = M, *sa = A, *sb = B, *dm = wM, *da = wA, *db = wB;
  for (int h = n >> 1; h >= 1; h >>= 1) {
    for (int i = threadIdx.x; i < h; i += kBlock) {
      const EnfRec r = enf_join(EnfRec{sm[2 * i], sa[2 * i], sb[2 * i]}, EnfRec{sm[2 * i + 1], sa[2 * i + 1], sb[2 * i + 1]});
      dm[i] = r.M; da[i] = r.a; db[i] = r.b;
    }
    __syncthreads();
    double* t;
    t = sm; sm = dm; dm = t;
    t = sa; sa = da; da = t;
    t = sb; sb = db; db = t;
  }
  const EnfRec r{sm[0], sa[0], sb[0]};
  __syncthreads();
  return r;
}

// One wave reduces n <= 256 ENF records (n a power of two) by the
// adjacent-pair tree: lane l first joins its aligned run of n/64 records,
// then lanes join in a butterfly over xor 1, 2, ..., min(n, 64)/2.  The join
// is commutative bit for bit, so lane l ^ d holds exactly the other half of
// every pair: the result is that of the adjacent-pair tree, in every lane
// l < n.  `rec(i)` yields record i.
template <class F>
__device__ __forceinline__ EnfRec wave_reduce_enf(int n, F rec) {
  const int lane = threadIdx.x & 63;
  EnfRec r{ninf(), 0.0, 0.0};
  if (n <= 64) {
    if (lane < n) r = rec(lane);
  } else if (n == 128) {
    r = enf_join(rec(2 * lane), rec(2 * lane + 1));
  } else {
    r = enf_join(enf_join(rec(4 * lane), rec(4 * lane + 1)), enf_join(rec(4 * lane + 2), rec(4 * lane + 3)));
  }
  const int width = n < 64 ? n : 64;
  for (int d = 1; d < width; d <<= 1) {
    const EnfRec o{__shfl_xor(r.M, d, 64), __shfl_xor(r.a, d, 64), __shfl_xor(r.b, d, 64)};
    r = enf_join(r, o);
  }
  return r;
}

// block-wide reductions with a fixed pattern (identical result in every block)
__device__ double block_max(double v, double* red) {
  for (int d = 1; d < 64; d <<= 1) v = fmax(v, __shfl_xor(v, d, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = red[0];
  for (int i = 1; i < kWaves; ++i) r = fmax(r, red[i]);
  __syncthreads();
  return r;
}

__device__ double block_sum(double v, double* red) {
  for (int d = 1; d < 64; d <<= 1) v += __shfl_xor(v, d, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = red[0];
  for (int i = 1; i < kWaves; ++i) r += red[i];
  __syncthreads();
  return r;
}

// log sum_i exp(scale * v[i]) over n values, whole block; `shared` says
// whether v lives in another block's published memory (device-scope reads)
__device__ double block_lse(const double* v, int n, double scale, double* red, bool shared) {
  double mx = ninf();
  for (int i = threadIdx.x; i < n; i += kBlock) mx = fmax(mx, scale * (shared ? get(v + i) : v[i]));
  mx = block_max(mx, red);
  if (mx == ninf()) return mx;
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += kBlock) s += dexp(scale * (shared ? get(v + i) : v[i]) - mx);
  s = block_sum(s, red);
  return mx + dlog(s);
}

}  // namespace airpf
