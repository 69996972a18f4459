// Device helpers shared by the filter kernels: cross-block memory accesses,
// the grid barrier, team (one island) and block reductions, the island
// pair-mean and pair-selection probability.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "dev_math.h"

namespace airpf {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;
constexpr int kMaxIslandsPerBlock = 256;   // the LDS plan of the forward kernel
constexpr int kPiCache = 4096;             // island maps the reverse kernel caches in LDS per step


__device__ __forceinline__ int64_t tree_off(int m, int level) {  // level >= 1
  return 2 * static_cast<int64_t>(m) - ((2 * static_cast<int64_t>(m)) >> (level - 1));
}

__device__ __forceinline__ double ninf() { return -__longlong_as_double(0x7ff0000000000000LL); }
template <typename R> __device__ __forceinline__ R neg_inf() {
  if constexpr (std::is_same<R, float>::value) return __uint_as_float(0xff800000u); else return ninf();
}
__device__ __forceinline__ double rmax(double a, double b) { return fmax(a, b); }
__device__ __forceinline__ float rmax(float a, float b) { return fmaxf(a, b); }

// log((exp(a) + exp(b)) / 2), symmetric in (a, b)
__device__ __forceinline__ double pair_mean(double a, double b) {
  const double hi = a > b ? a : b, lo = a > b ? b : a;
  double t = dexp(lo - hi);
  t = 1.0 + t;
  t = dlog(t);
  return hi == ninf() ? hi : (hi + t) - kLn2;
}

// log(exp(a) + exp(b)), symmetric in (a, b)
__device__ __forceinline__ double log_add_exp(double a, double b) {
  const double hi = a > b ? a : b, lo = a > b ? b : a;
  double t = dexp(lo - hi);
  t = 1.0 + t;
  t = dlog(t);
  return hi == ninf() ? hi : hi + t;
}

// probability that an island with log-weight lk takes its partner's block
__device__ __forceinline__ double take_partner_prob(double lk, double lp) {
  const double q = 1.0 / (1.0 + dexp(lk - lp));
  return lp == ninf() ? 0.0 : (lk == ninf() ? 1.0 : q);
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
// Split into its two halves so that a block can do work that does not
// depend on the other blocks between publishing its flag and waiting.
__device__ __forceinline__ void grid_arrive(unsigned* flags, int bid, unsigned& epoch) {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  ++epoch;
  if (threadIdx.x == 0) put(&flags[bid], epoch);
}

__device__ bool grid_wait(const unsigned* flags, int G, unsigned epoch, int* status) {
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

__device__ __forceinline__ bool grid_barrier(unsigned* flags, int G, int bid, unsigned& epoch, int* status) {
  grid_arrive(flags, bid, epoch);
  return grid_wait(flags, G, epoch, status);
}

// ------------------------------------------------------------ DPP lane moves
// Cross-lane moves inside a row of 16 lanes (and the two row broadcasts of
// the scan) through the VALU's data-parallel primitives, without the LDS
// crossbar.  Lanes a move does not write (masked rows, sources outside the
// row) read 0.  Controls: quad_perm(1,0,3,2) = 0xB1 and (2,3,0,1) = 0x4E
// (xor 1, xor 2), row_shr:k = 0x110 + k, row_mirror = 0x140 (lane i <- 15-i),
// row_half_mirror = 0x141 (i <- 7-i in each half row), row_bcast:15 = 0x142,
// row_bcast:31 = 0x143.
template <int CTRL, int ROWMASK = 0xf>
__device__ __forceinline__ uint32_t dpp32(uint32_t v) {
  return static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), CTRL, ROWMASK, 0xf, true));
}
template <int CTRL, int ROWMASK = 0xf>
__device__ __forceinline__ uint64_t dpp64(uint64_t v) {
  const uint32_t lo = dpp32<CTRL, ROWMASK>(static_cast<uint32_t>(v));
  const uint32_t hi = dpp32<CTRL, ROWMASK>(static_cast<uint32_t>(v >> 32));
  return (static_cast<uint64_t>(hi) << 32) | lo;
}
template <int CTRL>
__device__ __forceinline__ double dppd(double v) {
  return __longlong_as_double(static_cast<long long>(dpp64<CTRL>(static_cast<uint64_t>(__double_as_longlong(v)))));
}

// Lane l's value, in every lane (read through a scalar register).
__device__ __forceinline__ uint64_t readlane_u64(uint64_t v, int l) {
  const uint32_t lo = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(static_cast<uint32_t>(v)), l));
  const uint32_t hi = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(static_cast<uint32_t>(v >> 32)), l));
  return (static_cast<uint64_t>(hi) << 32) | lo;
}
__device__ __forceinline__ double readlane_f64(double v, int l) {
  return __longlong_as_double(static_cast<long long>(readlane_u64(static_cast<uint64_t>(__double_as_longlong(v)), l)));
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
  // partners xor 1, xor 2, then the mirrors of 8 and 16 lanes (each pairs a
  // lane with one holding the other half of its group), then xor 16, 32
  if (TP >= 2) v = fmax(v, dppd<0xB1>(v));
  if (TP >= 4) v = fmax(v, dppd<0x4E>(v));
  if (TP >= 8) v = fmax(v, dppd<0x141>(v));
  if (TP >= 16) v = fmax(v, dppd<0x140>(v));
  if (TP >= 64) {
    // whole wave: the four row maxima through scalar registers
    v = fmax(fmax(readlane_f64(v, 0), readlane_f64(v, 16)), fmax(readlane_f64(v, 32), readlane_f64(v, 48)));
  } else if (TP >= 32) {
    v = fmax(v, __shfl_xor(v, 16, 64));
  }
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

// the same tree for binary32 values (32-bit lane moves); `red` holds kWaves floats
__device__ __forceinline__ float readlane_f32(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
template <int CTRL>
__device__ __forceinline__ float dppf(float v) {
  return __uint_as_float(dpp32<CTRL>(__float_as_uint(v)));
}
__device__ __forceinline__ float team_max(float v, int TP, float* red) {
  if (TP >= 2) v = fmaxf(v, dppf<0xB1>(v));
  if (TP >= 4) v = fmaxf(v, dppf<0x4E>(v));
  if (TP >= 8) v = fmaxf(v, dppf<0x141>(v));
  if (TP >= 16) v = fmaxf(v, dppf<0x140>(v));
  if (TP >= 64) {
    v = fmaxf(fmaxf(readlane_f32(v, 0), readlane_f32(v, 16)), fmaxf(readlane_f32(v, 32), readlane_f32(v, 48)));
  } else if (TP >= 32) {
    v = fmaxf(v, __shfl_xor(v, 16, 64));
  }
  if (TP > 64) {
    const int tid = threadIdx.x;
    if ((tid & 63) == 0) red[tid >> 6] = v;
    __syncthreads();
    const int w0 = (tid / TP) * (TP >> 6);
    float r = red[w0];
    for (int i = 1; i < (TP >> 6); ++i) r = fmaxf(r, red[w0 + i]);
    __syncthreads();
    v = r;
  }
  return v;
}
__device__ __forceinline__ float team_max(float v, int TP, double* red) { return team_max(v, TP, reinterpret_cast<float*>(red)); }

__device__ __forceinline__ uint64_t team_sum_u64(uint64_t v, int TP, uint64_t* red) {
  if (TP >= 2) v += dpp64<0xB1>(v);
  if (TP >= 4) v += dpp64<0x4E>(v);
  if (TP >= 8) v += dpp64<0x141>(v);
  if (TP >= 16) v += dpp64<0x140>(v);
  if (TP >= 64) v = (readlane_u64(v, 0) + readlane_u64(v, 16)) + (readlane_u64(v, 32) + readlane_u64(v, 48));
  else if (TP >= 32) v += __shfl_xor(v, 16, 64);
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

// inclusive scan of v over the team's lanes (lane order): shifts by 1, 2, 4,
// 8 inside each row of 16 lanes, then the row totals carried forward by the
// two row broadcasts (lane 15 into the next row, lane 31 into rows 2 and 3)
__device__ __forceinline__ uint64_t team_scan_u64(uint64_t v, int TP, uint64_t* red) {
  const int tid = threadIdx.x;
  const int sl = tid & ((TP < 64 ? TP : 64) - 1);
  uint64_t t;
  if (TP > 1) { t = dpp64<0x111>(v); if (sl >= 1) v += t; }
  if (TP > 2) { t = dpp64<0x112>(v); if (sl >= 2) v += t; }
  if (TP > 4) { t = dpp64<0x114>(v); if (sl >= 4) v += t; }
  if (TP > 8) { t = dpp64<0x118>(v); if (sl >= 8) v += t; }
  if (TP > 16) v += dpp64<0x142, 0xa>(v);
  if (TP > 32) v += dpp64<0x143, 0xc>(v);
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

// DPP move of a 32-bit value where lanes without a source keep `old`
template <int CTRL, int ROWMASK = 0xf>
__device__ __forceinline__ int dpp_keep(int v, int old) {
  return __builtin_amdgcn_update_dpp(old, v, CTRL, ROWMASK, 0xf, false);
}

// Exclusive max-scan of an int over the team's lanes (lane order): the
// largest value of the lanes before this one, -1 for the team's first lane.
__device__ __forceinline__ int team_exclusive_max(int v, int TP, int* red) {
  const int tid = threadIdx.x;
  const int sl = tid & ((TP < 64 ? TP : 64) - 1);
  // inclusive within the wave part of the team: rows first, then the row broadcasts
  if (TP > 1) { const int t = dpp_keep<0x111>(v, -1); if (sl >= 1) v = v > t ? v : t; }
  if (TP > 2) { const int t = dpp_keep<0x112>(v, -1); if (sl >= 2) v = v > t ? v : t; }
  if (TP > 4) { const int t = dpp_keep<0x114>(v, -1); if (sl >= 4) v = v > t ? v : t; }
  if (TP > 8) { const int t = dpp_keep<0x118>(v, -1); if (sl >= 8) v = v > t ? v : t; }
  if (TP > 16) { const int t = dpp_keep<0x142, 0xa>(v, -1); v = v > t ? v : t; }
  if (TP > 32) { const int t = dpp_keep<0x143, 0xc>(v, -1); v = v > t ? v : t; }
  int wave_prev = -1;                          // the team's earlier waves (TP > 64)
  if (TP > 64) {
    if ((tid & 63) == 63) red[tid >> 6] = v;
    __syncthreads();
    const int w0 = (tid / TP) * (TP >> 6);
    for (int i = w0; i < (tid >> 6); ++i) wave_prev = wave_prev > red[i] ? wave_prev : red[i];
    __syncthreads();
    v = v > wave_prev ? v : wave_prev;
  }
  int ex = dpp_keep<0x138>(v, -1);             // wave_shr:1, lane l reads lane l-1
  if (sl == 0) ex = wave_prev;
  return ex;
}

// sum of a double over the team's lanes (fixed pattern; every lane gets it):
// partners xor 1, xor 2, the 8- and 16-lane mirrors, xor 16, xor 32 (each
// adds the other half of its group, so every lane holds the same bits)
__device__ __forceinline__ double team_sum_f64(double v, int TP, double* red) {
  if (TP >= 2) v += dppd<0xB1>(v);
  if (TP >= 4) v += dppd<0x4E>(v);
  if (TP >= 8) v += dppd<0x141>(v);
  if (TP >= 16) v += dppd<0x140>(v);
  if (TP >= 64) {
    // the rows' sums through scalar registers, in the tree xor 16, xor 32 forms
    v = (readlane_f64(v, 0) + readlane_f64(v, 16)) + (readlane_f64(v, 32) + readlane_f64(v, 48));
  } else if (TP >= 32) {
    v += __shfl_xor(v, 16, 64);
  }
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

// inclusive scan of a double over the team's lanes (lane order), in the
// pattern of team_scan_u64
__device__ __forceinline__ double team_scan_f64(double v, int TP, double* red) {
  const int tid = threadIdx.x;
  const int sl = tid & ((TP < 64 ? TP : 64) - 1);
  double t;
  if (TP > 1) { t = dppd<0x111>(v); if (sl >= 1) v += t; }
  if (TP > 2) { t = dppd<0x112>(v); if (sl >= 2) v += t; }
  if (TP > 4) { t = dppd<0x114>(v); if (sl >= 4) v += t; }
  if (TP > 8) { t = dppd<0x118>(v); if (sl >= 8) v += t; }
  if (TP > 16) v += __longlong_as_double(static_cast<long long>(dpp64<0x142, 0xa>(static_cast<uint64_t>(__double_as_longlong(v)))));
  if (TP > 32) v += __longlong_as_double(static_cast<long long>(dpp64<0x143, 0xc>(static_cast<uint64_t>(__double_as_longlong(v)))));
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

// ENF sums of a set of island log-weights L.  The record (E, a, b) holds
// a = sum exp(L) 2^-E and b = sum exp(2L) 2^-2E for an integer E kept as a
// double (E = -inf for an empty or all-dead set).  A leaf takes E as the
// integer nearest L / log 2, so its share exp(L - E log 2) lies in
// [0.7, 1.42]; two records join at the larger E with exact power-of-two
// rescaling (two ldexp and one addition per sum, no exponential).  The ENF
// (m^-1 sum W)^2 / (m^-1 sum W^2) is a^2 / b up to the block factors: 2^E
// cancels.  When one member's weight swamps the others' below rounding, a
// and b reduce to that member's w and fl(w^2) and the ENF lands exactly on
// its rational value, as the definition does.
struct EnfRec { double E, a, b; };

__device__ __forceinline__ EnfRec enf_leaf(double L) {
  const bool dead = L == ninf();
  const double E = dead ? 0.0 : rint(L * kInvLn2);
  const double w = dexp(fma(-E, kLn2Tail, fma(-E, kLn2Head, dead ? 0.0 : L)));
  return dead ? EnfRec{L, 0.0, 0.0} : EnfRec{E, w, w * w};
}

// Branch-free: an empty side (E = -inf, a = b = 0) contributes exact zeros.
__device__ __forceinline__ EnfRec enf_join(const EnfRec& x, const EnfRec& y) {
  const double E = x.E > y.E ? x.E : y.E;
  // exponent gaps <= 0, clamped (an empty side's gap is -inf or NaN)
  const int dx = static_cast<int>(fmax(x.E - E, -4000.0)), dy = static_cast<int>(fmax(y.E - E, -4000.0));
  return EnfRec{E, __builtin_ldexp(x.a, dx) + __builtin_ldexp(y.a, dy),
                __builtin_ldexp(x.b, 2 * dx) + __builtin_ldexp(y.b, 2 * dy)};
}

// Whether the stage's ENF am^2 / bm lies below tau, decided as the rounded
// quotient decides it.  Far from the threshold the product tau * bm settles
// it (a relative margin of 2^-40 covers the roundings of both sides); only
// within the margin is the division done.  bm = 0 (NaN or infinite
// quotient) is never below.
__device__ __forceinline__ bool enf_below(double am, double bm, double tau) {
  const double num = am * am, lim = tau * bm;
  if (num < lim * (1.0 - 0x1p-40)) return true;
  if (num > lim * (1.0 + 0x1p-40)) return false;
  return num / bm < tau;
}

// One wave reduces n <= 1024 ENF records (n a power of two) by the
// adjacent-pair tree: lane l first joins its aligned run of n/64 records,
// then lanes join in a butterfly over groups of 2, 4, ..., min(n, 64).  The
// join is commutative bit for bit and a lane's partner holds exactly the
// other half of its group, so the result is that of the adjacent-pair tree,
// in every lane l < n.  `rec(i)` yields record i.
// The lanes' part of wave_reduce_enf: lane l holds the record of its
// aligned run; groups of 2, 4, ..., min(n, 64) lanes join (xor 1, xor 2,
// then the 8- and 16-lane mirrors, whose partner holds exactly the other
// half of the group as with xor 4, xor 8, then xor 16, xor 32; a whole wave
// joins its four rows' records through scalar registers in that same tree).
__device__ __forceinline__ EnfRec wave_butterfly_enf(EnfRec r, int n) {
  if (n >= 2) r = enf_join(r, EnfRec{dppd<0xB1>(r.E), dppd<0xB1>(r.a), dppd<0xB1>(r.b)});
  if (n >= 4) r = enf_join(r, EnfRec{dppd<0x4E>(r.E), dppd<0x4E>(r.a), dppd<0x4E>(r.b)});
  if (n >= 8) r = enf_join(r, EnfRec{dppd<0x141>(r.E), dppd<0x141>(r.a), dppd<0x141>(r.b)});
  if (n >= 16) r = enf_join(r, EnfRec{dppd<0x140>(r.E), dppd<0x140>(r.a), dppd<0x140>(r.b)});
  auto row = [&](int l) { return EnfRec{readlane_f64(r.E, l), readlane_f64(r.a, l), readlane_f64(r.b, l)}; };
  if (n >= 64) {
    // rows (0, 1) and (2, 3), then the two halves: the tree xor 16, xor 32 forms
    r = enf_join(enf_join(row(0), row(16)), enf_join(row(32), row(48)));
  } else if (n >= 32) {
    r = enf_join(r, EnfRec{__shfl_xor(r.E, 16, 64), __shfl_xor(r.a, 16, 64), __shfl_xor(r.b, 16, 64)});
  }
  return r;
}

// The join of the n records of a wave (n <= 256 a power of two; lane l
// holds records per*l .. per*l + per - 1, per = max(1, n/64) <= 4, the rest
// empty) over the adjacent-pair tree, in one rescaling: every record is
// brought to the largest E of all, then a and b are summed over the same
// tree as wave_butterfly_enf.  The result equals the pairwise joins bit for
// bit: scaling by a power of two commutes with each rounded sum while the
// values stay normal, and a term scaled below 2^-1000 of the largest is
// lost below rounding either way (up to the rounding of such a subnormal
// term).  Every lane gets the record.
__device__ __forceinline__ EnfRec wave_join_flat(const EnfRec* rec, int per, int n) {
  double e = rec[0].E;
  if (per >= 2) e = fmax(e, rec[1].E);
  if (per >= 4) e = fmax(e, fmax(rec[2].E, rec[3].E));
  e = fmax(e, dppd<0xB1>(e));
  e = fmax(e, dppd<0x4E>(e));
  e = fmax(e, dppd<0x141>(e));
  e = fmax(e, dppd<0x140>(e));
  e = fmax(fmax(readlane_f64(e, 0), readlane_f64(e, 16)), fmax(readlane_f64(e, 32), readlane_f64(e, 48)));
  double A[4], B[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int g = static_cast<int>(fmax(rec[j].E - e, -4000.0));     // an empty record's gap is -inf or NaN
    A[j] = __builtin_ldexp(rec[j].a, g);
    B[j] = __builtin_ldexp(rec[j].b, 2 * g);
  }
  double a = per == 4 ? (A[0] + A[1]) + (A[2] + A[3]) : (per == 2 ? A[0] + A[1] : A[0]);
  double b = per == 4 ? (B[0] + B[1]) + (B[2] + B[3]) : (per == 2 ? B[0] + B[1] : B[0]);
  const int nl = n >= 64 ? 64 : n;                                  // lanes holding records
  if (nl >= 2) { a += dppd<0xB1>(a); b += dppd<0xB1>(b); }
  if (nl >= 4) { a += dppd<0x4E>(a); b += dppd<0x4E>(b); }
  if (nl >= 8) { a += dppd<0x141>(a); b += dppd<0x141>(b); }
  if (nl >= 16) { a += dppd<0x140>(a); b += dppd<0x140>(b); }
  if (nl >= 64) {
    a = (readlane_f64(a, 0) + readlane_f64(a, 16)) + (readlane_f64(a, 32) + readlane_f64(a, 48));
    b = (readlane_f64(b, 0) + readlane_f64(b, 16)) + (readlane_f64(b, 32) + readlane_f64(b, 48));
  } else if (nl >= 32) {
    a += __shfl_xor(a, 16, 64);
    b += __shfl_xor(b, 16, 64);
    a = readlane_f64(a, 0);
    b = readlane_f64(b, 0);
  } else {
    a = readlane_f64(a, 0);
    b = readlane_f64(b, 0);
  }
  return EnfRec{e, a, b};
}

template <class F>
__device__ __forceinline__ EnfRec wave_reduce_enf(int n, F rec) {
  const int lane = threadIdx.x & 63;
  EnfRec r{ninf(), 0.0, 0.0};
  if (n <= 64) {
    if (lane < n) r = rec(lane);
  } else {
    // the lane's run of per = n/64 records (2 to 16) by the adjacent-pair
    // tree, kept as a binary counter: after record j, the partial of the
    // aligned group of 2^t records ending at j is complete for every t with
    // bit t of j + 1 clear below it
    const int per = n >> 6;
    EnfRec s1{ninf(), 0.0, 0.0}, s2 = s1, s4 = s1, s8 = s1, s16 = s1;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      if (j < per) {
        EnfRec x = rec(per * lane + j);
        if ((j & 1) == 0) { s1 = x; continue; }
        x = enf_join(s1, x);
        if ((j & 2) == 0) { s2 = x; continue; }
        x = enf_join(s2, x);
        if ((j & 4) == 0) { s4 = x; continue; }
        x = enf_join(s4, x);
        if ((j & 8) == 0) { s8 = x; continue; }
        s16 = enf_join(s8, x);
      }
    }
    r = per == 2 ? s2 : (per == 4 ? s4 : (per == 8 ? s8 : s16));
  }
  return wave_butterfly_enf(r, n);
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
