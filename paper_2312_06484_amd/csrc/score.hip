// Adjoint of the AIRPF filter for the score d log Zhat / d theta (not part
// of the paper: the estimator differentiated here is the path-space one).
//
// With the noise and every discrete decision of the forward run held fixed,
// the path-space score is
//   G = sum over final particles of Wbar_i * (d/dtheta of the sum of log g
//       along particle i's ancestral path, x reparameterised by its noise).
// Reverse accumulation over steps n = T-1 .. 0, per particle (k, i):
//   D_n(k,i)  = final weight carried by the descendants of (k,i):
//               D_{T-1} = Wbar;  D_n(k,i) = sum over children (k', j) of D_{n+1}(k', j)
//   lam_n(k,i) = D_n(k,i) dlw/dx (x_n^{k,i}) + sum_children (dF/dx)^T lam_{n+1}(k', j)
//   G += D_n dlogg/dtheta + sum over mutations lam_{n+1} . dF/dtheta + lam_0 . dx_0/dtheta
// The pathwise seed (the derivative of the run's own log Zhat with every
// decision held fixed) replaces D_n by the adjoint of log g_n(x_n^{k,i})
// through the island weights: with nu_{n,k} = d log Zhat / d L_{n,k}, L_{n,k}
// island k's log-weight after step n's weighting,
//   D_n(k,i)  = nu_{n,k} softmax_i(log g_n^{k,.}),
//   nu_{n,k}  = (sum of nu_{n+1,k'} over k's aligned 2^{s*_n}-block) W_{n,k} / (block's sum of W_n)
// (the entering weight of step n+1 is the block mean of the W_n, the
// composite of the stages' pair means), nu_{T-1,k} = W_{T-1,k} / sum W_{T-1};
// lam and the theta terms follow as above.  At T-1 both seeds coincide.
// Children of (n, k, i): slots j of islands k' with pi_n(k') = k and
// a_{n,k}(j) = i.  The islands with pi_n(k') = k all lie in k's aligned
// 2^{s*_n}-block, so each source island scans that block (ballot, ascending
// order); within the island the ancestors are sorted, so the slots of one
// particle form a run and their sums come from one prefix sum.  Nothing is
// accumulated with atomics: the result is bit-reproducible.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dev_models.h"
#include "dev_sync.h"
#include "internal.h"

namespace airpf {

// Sums acc[0..63] over the 64 lanes of a wave, lane l returning the total of
// acc[l]: at each level a lane keeps the half of its values indexed by its
// own lane bit and adds the partner's copy of that half (xor 32, 16, 8, 4,
// 2, 1), 63 exchanges instead of 64 full reductions.  The pattern is fixed.
__device__ __forceinline__ double wave_reduce_scatter64(double (&acc)[64]) {
  const int l = threadIdx.x & 63;
#pragma unroll
  for (int i = 0; i < 32; ++i) {
    const bool h = (l & 32) != 0;
    const double send = h ? acc[i] : acc[i + 32], keep = h ? acc[i + 32] : acc[i];
    acc[i] = keep + __shfl_xor(send, 32, 64);
  }
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const bool h = (l & 16) != 0;
    const double send = h ? acc[i] : acc[i + 16], keep = h ? acc[i + 16] : acc[i];
    acc[i] = keep + __shfl_xor(send, 16, 64);
  }
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const bool h = (l & 8) != 0;
    const double send = h ? acc[i] : acc[i + 8], keep = h ? acc[i + 8] : acc[i];
    acc[i] = keep + dppd<0x128>(send);              // row_ror:8 = xor 8 inside a row
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const bool h = (l & 4) != 0;
    const double send = h ? acc[i] : acc[i + 4], keep = h ? acc[i + 4] : acc[i];
    acc[i] = keep + __shfl_xor(send, 4, 64);
  }
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const bool h = (l & 2) != 0;
    const double send = h ? acc[i] : acc[i + 2], keep = h ? acc[i + 2] : acc[i];
    acc[i] = keep + dppd<0x4E>(send);
  }
  {
    const bool h = (l & 1) != 0;
    const double send = h ? acc[0] : acc[1], keep = h ? acc[1] : acc[0];
    acc[0] = keep + dppd<0xB1>(send);
  }
  return acc[0];
}

// The same reduce-scatter of acc[8i + c] = sum_r u[r][i] v[r][c] (64 entries,
// an 8 x 8 outer product summed over the lane's slots), with the first
// level's values formed as they are exchanged: only the 32 entries a lane
// keeps are ever held at once.
template <int PPT>
__device__ __forceinline__ double wave_reduce_scatter64_outer(const double (&u)[PPT][9], const double (&v)[PPT][8]) {
  const int l = threadIdx.x & 63;
  const bool h = (l & 32) != 0;
  double acc[64];
#pragma unroll
  for (int i = 0; i < 32; ++i) {
    double lo = 0.0, hi = 0.0;
#pragma unroll
    for (int r = 0; r < PPT; ++r) {
      lo += u[r][i >> 3] * v[r][i & 7];
      hi += u[r][(i + 32) >> 3] * v[r][(i + 32) & 7];
    }
    const double send = h ? lo : hi, keep = h ? hi : lo;
    acc[i] = keep + __shfl_xor(send, 32, 64);
  }
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const bool g = (l & 16) != 0;
    const double send = g ? acc[i] : acc[i + 16], keep = g ? acc[i + 16] : acc[i];
    acc[i] = keep + __shfl_xor(send, 16, 64);
  }
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const bool g = (l & 8) != 0;
    const double send = g ? acc[i] : acc[i + 8], keep = g ? acc[i + 8] : acc[i];
    acc[i] = keep + dppd<0x128>(send);
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const bool g = (l & 4) != 0;
    const double send = g ? acc[i] : acc[i + 4], keep = g ? acc[i + 4] : acc[i];
    acc[i] = keep + __shfl_xor(send, 4, 64);
  }
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const bool g = (l & 2) != 0;
    const double send = g ? acc[i] : acc[i + 2], keep = g ? acc[i + 2] : acc[i];
    acc[i] = keep + dppd<0x4E>(send);
  }
  {
    const bool g = (l & 1) != 0;
    const double send = g ? acc[0] : acc[1], keep = g ? acc[1] : acc[0];
    acc[0] = keep + dppd<0xB1>(send);
  }
  return acc[0];
}

template <class Model, typename Store, int PPT>
__device__ __forceinline__ void backward_body(const BwdArgs& a, const int bid) {
  constexpr int DX = Model::DX;
  constexpr int NZ = PPT * DX;
  constexpr int P = Model::P;
  constexpr int NV = DX + 1;                   // per slot: lam (DX) and D
  static_assert(NZ % 4 == 0, "a lane consumes whole Philox blocks");
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double red_d[kWaves];

  const int tid = threadIdx.x;
  const int TP = a.TP, tpb = kBlock / TP;
  const int team = tid / TP, lane = tid & (TP - 1);
  const int m = a.m, N = a.N, c = a.c;
  const int kbase = bid * c;
  const Key key = make_key(a.seed);
  const int passes = (c + tpb - 1) / tpb;

  Store* sx = reinterpret_cast<Store*>(smem);                                        // [kBlock*NZ]
  double* sP = reinterpret_cast<double*>(smem + ((sizeof(Store) * kBlock * NZ + 15) & ~size_t(15)));  // [kBlock*PPT*NV]
  int* sA = reinterpret_cast<int*>(sP + kBlock * PPT * NV);                          // [kBlock*PPT]
  int* sS = sA + kBlock * PPT;                                                       // [kBlock*PPT] run start
  int* sE = sS + kBlock * PPT;                                                       // [kBlock*PPT] run end
  int* s_pi = sE + kBlock * PPT;                                                     // [kPiCache] island maps

  unsigned epoch = 0;
  const double logz = *a.logz;

  for (int64_t n = a.n_hi - 1; n >= a.n_lo; --n) {
    // the children of step n's particles are in their island's aligned
    // 2^{s*_n}-block, and step n overwrites the adjoints that step n+1 read
    // from the 2^{s*_{n+1}}-blocks of its own children: when both stay inside
    // this block (s* <= log2 c), the block barrier orders every access
    if (n < a.n_hi - 1) {
      const bool cross_next = n + 1 < a.T - 1 && a.sstar_all[n + 1] > a.lc;
      if (a.sstar_all[n] > a.lc || cross_next) {
        if (!grid_barrier(a.bar, a.G, bid, epoch, a.status)) return;
      } else {
        __syncthreads();
      }
    }
    const bool last = (n == a.T - 1);
    const int B = last ? 1 : (1 << a.sstar_all[n]);
    const int par = static_cast<int>(n & 1), npar = par ^ 1;
    const double* yn = a.y + n * a.dy;
    // the island maps of step n over the candidates of this block's islands
    // (the aligned 2^{s*}-block of each), cached in LDS when they fit
    const int R_len = B > c ? B : c;
    const int R_lo = kbase & ~(B - 1);
    const bool pi_cached = !last && R_len <= kPiCache;
    if (pi_cached) {
      for (int i = tid; i < R_len; i += kBlock) s_pi[i] = a.pi_all[n * m + R_lo + i];
      __syncthreads();
    }

    for (int p = 0; p < passes; ++p) {
      const int li = p * tpb + team;
      const bool active = li < c;
      const int k = kbase + (active ? li : 0);
      const int j0 = lane * PPT;
      Store* sxt = sx + team * TP * NZ;
      double* sPt = sP + team * TP * PPT * NV;
      int* sAt = sA + team * TP * PPT;
      int* sSt = sS + team * TP * PPT;
      int* sEt = sE + team * TP * PPT;
      double acc[P];                             // this island's contribution at step n
#pragma unroll
      for (int q = 0; q < P; ++q) acc[q] = 0.0;

      // ---- the state entering step n and its per-particle log-potential ----
      const Store* xs = static_cast<const Store*>(a.rec_x) + ((n - a.n_lo) * m + k) * static_cast<int64_t>(N) * DX;
      double x[PPT][DX], lw[PPT];
#pragma unroll
      for (int r = 0; r < PPT; ++r) {
        const bool valid = active && (j0 + r < N);
        Store xr[DX];
#pragma unroll
        for (int d = 0; d < DX; ++d) {
          const Store v = valid ? xs[(j0 + r) * DX + d] : Store(0);
          xr[d] = v;
          x[r][d] = static_cast<double>(v);
          sxt[(j0 + r) * DX + d] = v;
        }
        // log g in the particles' precision, as the forward pass weighted them
        Store v = valid ? Model::template logpot<Store>(a.mp, xr, yn) : neg_inf<Store>();
        if (!(v == v)) v = neg_inf<Store>();
        lw[r] = static_cast<double>(v);
      }

      double lam[PPT][DX], D[PPT];
#pragma unroll
      for (int r = 0; r < PPT; ++r) {
        D[r] = 0.0;
#pragma unroll
        for (int d = 0; d < DX; ++d) lam[r][d] = 0.0;
      }
      double sl[PPT][NV];                        // per slot: sum over children of (lam, D)
      double xp[PPT][DX];                        // parent value of each slot: x_n[k][a(j)]
#pragma unroll
      for (int r = 0; r < PPT; ++r) {
#pragma unroll
        for (int v = 0; v < NV; ++v) sl[r][v] = 0.0;
#pragma unroll
        for (int d = 0; d < DX; ++d) xp[r][d] = 0.0;
      }

      if (last) {
        // final normalised weights: Wbar = exp(Lpre_k + log g - log(m N) - log Zhat)
        const double lpre = a.lpre_all[n * m + k];
#pragma unroll
        for (int r = 0; r < PPT; ++r)
          D[r] = (active && j0 + r < N && lw[r] != ninf()) ? dexp(lpre + lw[r] + a.c_log - a.log_mN - logz) : 0.0;
      } else {
        // ancestors of this island's slots at step n
        const uint16_t* an = a.rec_anc + ((n - a.n_lo) * m + k) * static_cast<int64_t>(N);
#pragma unroll
        for (int r = 0; r < PPT; ++r) sAt[j0 + r] = (active && j0 + r < N) ? static_cast<int>(an[j0 + r]) : 0x7fffffff;
        team_sync(TP);

#pragma unroll
        for (int r = 0; r < PPT; ++r)
#pragma unroll
          for (int d = 0; d < DX; ++d)
            xp[r][d] = (active && j0 + r < N) ? static_cast<double>(sxt[sAt[j0 + r] * DX + d]) : 0.0;

        // ---- children: islands k' of k's 2^{s*}-block with pi_n(k') = k ----
        const int W = TP < 64 ? TP : 64;
        const int sl_lane = TP < 64 ? lane : (tid & 63);
        const int seg0 = TP < 64 ? ((tid & 63) & ~(TP - 1)) : 0;
        const int blo = k & ~(B - 1);
        const Store* lam_in = static_cast<const Store*>(a.lam[npar]);
        const Store* del_in = static_cast<const Store*>(a.del[npar]);
        double nu_acc = 0.0;                     // pathwise: this lane's part of the block sum of nu_{n+1}
        for (int it = 0; it < B; it += W) {
          const int cand = blo + it + sl_lane;
          if (a.pathwise && active && it + sl_lane < B) nu_acc += get(a.nu[npar] + cand);
          const bool match = active && (it + sl_lane < B) &&
                             (pi_cached ? s_pi[cand - R_lo] : a.pi_all[n * m + cand]) == k;
          const unsigned long long ball = __ballot(match);
          unsigned long long seg = (W == 64) ? ball : ((ball >> seg0) & ((1ull << W) - 1));
          while (seg) {
            const int b = __builtin_ctzll(seg);
            seg &= seg - 1;
            const int child = blo + it + b;
            double z[NZ];
            for (int g = 0; g < NZ / 4; ++g) {
              Store t[4];
              normals4(key, static_cast<uint32_t>((j0 * DX) / 4 + g), static_cast<uint32_t>(child),
                       static_cast<uint32_t>(n + 1), t);
#pragma unroll
              for (int q = 0; q < 4; ++q) z[4 * g + q] = t[q];
            }
#pragma unroll
            for (int r = 0; r < PPT; ++r) {
              const int j = j0 + r;
              if (j < N) {
                double lc[DX];
#pragma unroll
                for (int d = 0; d < DX; ++d) {
                  lc[d] = static_cast<double>(get(lam_in + (static_cast<int64_t>(child) * N + j) * DX + d));
                  sl[r][d] += lc[d];
                }
                sl[r][DX] += static_cast<double>(get(del_in + static_cast<int64_t>(child) * N + j));
                if constexpr (!Model::kThetaOuter) Model::prop_vjp_theta(a.mp, xp[r], z + r * DX, lc, acc);
              }
            }
          }
        }

        // ---- back through the internal resampling: runs of equal ancestors ----
        // Multinomial draws leave the ancestors in no order: the slots are
        // sorted by (ancestor, slot) first (a bitonic sort of the team's keys
        // in LDS; keys are distinct, so the order is fixed), and the runs are
        // taken over the sorted slots, each slot's sums moved to its sorted
        // position.
        bool sorted_slots = false;
        {
          if (a.multinomial) {
            constexpr int kNoKey = 0x7fffffff;
#pragma unroll
            for (int r = 0; r < PPT; ++r) {
              const int j = j0 + r;
              const int aj = sAt[j];
              sAt[j] = (active && j < N) ? ((aj << 11) | j) : kNoKey;
#pragma unroll
              for (int v = 0; v < NV; ++v) sPt[j * NV + v] = sl[r][v];
            }
            team_sync(TP);
            const int np = TP * PPT;
            for (int kk = 2; kk <= np; kk <<= 1) {
              for (int jj = kk >> 1; jj > 0; jj >>= 1) {
                for (int t = lane; t < np / 2; t += TP) {
                  const int i0 = (t / jj) * 2 * jj + (t % jj), i1 = i0 + jj;
                  const int k0 = sAt[i0], k1 = sAt[i1];
                  if ((k0 > k1) == ((i0 & kk) == 0)) { sAt[i0] = k1; sAt[i1] = k0; }
                }
                team_sync(TP);
              }
            }
#pragma unroll
            for (int r = 0; r < PPT; ++r) {
              const int key = sAt[j0 + r];
              const int js = key & 2047;
#pragma unroll
              for (int v = 0; v < NV; ++v) sl[r][v] = key != kNoKey ? sPt[js * NV + v] : 0.0;
            }
            team_sync(TP);
            sorted_slots = true;
          }
        }
        auto anc_at = [&](int j) { return sorted_slots ? (sAt[j] >> 11) : sAt[j]; };
        double run_v[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) run_v[v] = 0.0;
#pragma unroll
        for (int r = 0; r < PPT; ++r)
#pragma unroll
          for (int v = 0; v < NV; ++v) run_v[v] += sl[r][v];
        double base[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) base[v] = team_scan_f64(run_v[v], TP, red_d) - run_v[v];
#pragma unroll
        for (int r = 0; r < PPT; ++r) {
          sSt[j0 + r] = -1;
#pragma unroll
          for (int v = 0; v < NV; ++v) {
            base[v] += sl[r][v];
            sPt[(j0 + r) * NV + v] = base[v];          // inclusive prefix over slots
          }
        }
        team_sync(TP);
#pragma unroll
        for (int r = 0; r < PPT; ++r) {
          const int j = j0 + r;
          if (active && j < N) {
            const int aj = anc_at(j);
            if (j == 0 || anc_at(j - 1) != aj) sSt[aj] = j;
            if (j == N - 1 || anc_at(j + 1) != aj) sEt[aj] = j;
          }
        }
        team_sync(TP);
#pragma unroll
        for (int r = 0; r < PPT; ++r) {
          const int i = j0 + r;
          if (active && i < N && sSt[i] >= 0) {
            const int s0 = sSt[i], e0 = sEt[i];
            double tot[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) tot[v] = sPt[e0 * NV + v] - (s0 > 0 ? sPt[(s0 - 1) * NV + v] : 0.0);
            Model::prop_vjp_x(a.mp, tot, lam[r]);
            D[r] = tot[DX];
            if constexpr (Model::kThetaOuter) {
              // sorted slots: the outer products below are taken per parent,
              // its children's sums with its own state (the same sum grouped
              // by parent)
              if (sorted_slots) {
#pragma unroll
                for (int v = 0; v < NV; ++v) sl[r][v] = tot[v];
              }
            }
          } else if (sorted_slots) {
#pragma unroll
            for (int v = 0; v < NV; ++v) sl[r][v] = 0.0;          // a parent without children
          }
          if constexpr (Model::kThetaOuter) {
            if (sorted_slots) {
#pragma unroll
              for (int d = 0; d < DX; ++d) xp[r][d] = (active && i < N) ? x[r][d] : 0.0;
            }
          }
        }
        if (a.pathwise) {
          // D_n(k,i) = (block sum of nu_{n+1}) W_{n,k} softmax_i / (block sum of W_n):
          // exp(Lpre_{n,k} + log g_i - log N - Lpre_{n+1,k} - s* log 2), the block
          // mean of the W_n being the entering weight of step n+1
          const double nuB = team_sum_f64(nu_acc, W, red_d);
          const double lpre = a.lpre_all[n * m + k], lnext = a.lpre_all[(n + 1) * m + k];
          const double sh = a.c_log - a.log_N - lnext - static_cast<double>(a.sstar_all[n]) * kLn2;
#pragma unroll
          for (int r = 0; r < PPT; ++r)
            D[r] = (active && j0 + r < N && lw[r] != ninf() && lpre != ninf() && lnext != ninf())
                       ? nuB * dexp((lpre + lw[r]) + sh) : 0.0;
        }
      }
      if (a.pathwise) {
        // nu_{n,k} = sum_i D_n(k,i), read by step n-1
        double dsum = 0.0;
#pragma unroll
        for (int r = 0; r < PPT; ++r) dsum += D[r];
        dsum = team_sum_f64(dsum, TP, red_d);
        if (lane == 0 && active) put(a.nu[par] + k, dsum);
      }

      // ---- the weighting terms of step n ----
#pragma unroll
      for (int r = 0; r < PPT; ++r) {
        if (active && j0 + r < N && D[r] != 0.0) {
          double gx[DX];
          Model::dlogpot_dx(a.mp, x[r], yn, gx);
#pragma unroll
          for (int d = 0; d < DX; ++d) lam[r][d] += D[r] * gx[d];
          Model::dlogpot_dtheta(a.mp, x[r], yn, D[r], acc);
        }
      }
      if (n == 0) {
        double z[NZ];
        for (int g = 0; g < NZ / 4; ++g) {
          Store t[4];
          normals4(key, static_cast<uint32_t>((j0 * DX) / 4 + g), static_cast<uint32_t>(k), 0u, t);
#pragma unroll
          for (int q = 0; q < 4; ++q) z[4 * g + q] = t[q];
        }
#pragma unroll
        for (int r = 0; r < PPT; ++r)
          if (active && j0 + r < N) Model::init_vjp_theta(a.mp, z + r * DX, lam[r], acc);
      } else if (active) {
        Store* lo = static_cast<Store*>(a.lam[par]) + static_cast<int64_t>(k) * N * DX;
        Store* dl = static_cast<Store*>(a.del[par]) + static_cast<int64_t>(k) * N;
#pragma unroll
        for (int r = 0; r < PPT; ++r) {
          const int i = j0 + r;
          if (i < N) {
#pragma unroll
            for (int d = 0; d < DX; ++d) put(lo + i * DX + d, static_cast<Store>(lam[r][d]));
            put(dl + i, static_cast<Store>(D[r]));
          }
        }
      }
      // the island's gradient contribution, summed over its lanes in a fixed
      // pattern and added to the island's own accumulator (in step order)
      bool summed = false;
      if constexpr (Model::kThetaOuter && P == 64 && DX == 8) {
        if (TP == 64) {
          const double v = wave_reduce_scatter64_outer<PPT>(sl, xp);
          if (active) a.gisl[static_cast<int64_t>(k) * P + (tid & 63)] += v;
          summed = true;
        }
      } else if constexpr (P == 64) {
        if (TP == 64) {
          const double v = wave_reduce_scatter64(acc);
          if (active) a.gisl[static_cast<int64_t>(k) * P + (tid & 63)] += v;
          summed = true;
        }
      }
      if constexpr (Model::kThetaOuter) {
        // the outer products of the slots, where the fused path above did not run
        if (!summed) {
#pragma unroll
          for (int r = 0; r < PPT; ++r)
#pragma unroll
            for (int i = 0; i < DX; ++i)
#pragma unroll
              for (int c2 = 0; c2 < DX; ++c2) acc[i * DX + c2] += sl[r][i] * xp[r][c2];
        }
      }
      if (!summed) {
#pragma unroll
        for (int q = 0; q < P; ++q) {
          const double v = team_sum_f64(acc[q], TP, red_d);
          if (lane == 0 && active) a.gisl[static_cast<int64_t>(k) * P + q] += v;
        }
      }
      team_sync(TP);
    }
  }
}

template <class Model, typename Store, int PPT>
__global__ __launch_bounds__(kBlock) void backward_kernel(BwdArgs a) {
  backward_body<Model, Store, PPT>(a, static_cast<int>(blockIdx.x));
}

// three waves per SIMD for the batch of models with a state of one, two or
// four dimensions (VGPRs capped at 168, at most a few spilled): the reverse
// pass of many problems is limited by latency, not by registers.  The others
// take two (the cap spilled dozens to hundreds of registers to scratch for
// d_x = 3 and 8).
template <class Model, typename Store, int PPT>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(3, 3))) void backward_batch_kernel(const BwdArgs* probs, const int2* bmap) {
  const int2 pb = bmap[blockIdx.x];
  backward_body<Model, Store, PPT>(probs[pb.x], pb.y);
}
template <class Model, typename Store, int PPT>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2, 2))) void backward_batch_kernel_wide(const BwdArgs* probs, const int2* bmap) {
  const int2 pb = bmap[blockIdx.x];
  backward_body<Model, Store, PPT>(probs[pb.x], pb.y);
}

// grad[q] = sum over islands of gisl[k*P + q]: lane t adds islands
// [t m/256, (t+1) m/256) in order, then the 256 partials by adjacent pairs.
// The order depends on m only.
__global__ __launch_bounds__(kBlock) void island_grad_sum_kernel(const double* gisl, int m, int P, double* out) {
  __shared__ double v[kBlock];
  __shared__ double w[kBlock / 2];
  const int per = (m + kBlock - 1) / kBlock;
  for (int q = 0; q < P; ++q) {
    double acc = 0.0;
    for (int i = threadIdx.x * per; i < (threadIdx.x + 1) * per && i < m; ++i) acc += gisl[static_cast<int64_t>(i) * P + q];
    v[threadIdx.x] = acc;
    __syncthreads();
    double* src = v;
    double* dst = w;
    for (int h = kBlock / 2; h >= 1; h >>= 1) {
      if (threadIdx.x < h) dst[threadIdx.x] = src[2 * threadIdx.x] + src[2 * threadIdx.x + 1];
      __syncthreads();
      double* t = src; src = dst; dst = t;
    }
    if (threadIdx.x == 0) out[q] = src[0];
    __syncthreads();
  }
}

// ============================================================ host launcher

static int pow2_ceil_b(int v) { int p = 1; while (p < v) p <<= 1; return p; }

static size_t bwd_smem_bytes(size_t store_bytes, int ppt, int dx) {
  const size_t sx = (store_bytes * kBlock * ppt * dx + 15) & ~size_t(15);
  return sx + 8 * size_t(kBlock) * ppt * (dx + 1) + 3 * 4 * size_t(kBlock) * ppt + 4 * size_t(kPiCache);
}

template <class Model, typename Store, int PPT>
static hipError_t launch_b(const FwdLaunch& L, const BwdArgs& a0, int* plan_p) {
  BwdArgs a = a0;
  auto kern = backward_kernel<Model, Store, PPT>;
  const size_t smem = bwd_smem_bytes(sizeof(Store), PPT, Model::DX);
  if (plan_p) {
    // the block count must be the forward plan's (same islands per block)
    int per_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, kBlock, smem);
    if (e != hipSuccess) return e;
    *plan_p = per_cu * L.num_cus;
    return hipSuccess;
  }
  a.TP = pow2_ceil_b((a.N + PPT - 1) / PPT);
  void* args[] = {&a};
  return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(kern), dim3(a.G), dim3(kBlock), args,
                                    static_cast<unsigned>(smem), L.stream);
}

// same particles-per-lane choice as the forward launcher
template <class Model, typename Store>
static hipError_t dispatch_b(const FwdLaunch& L, const BwdArgs& a, int* plan_p) {
  constexpr int DX = Model::DX;
  if constexpr (DX % 4 == 0) {
    if (a.N <= 256) return launch_b<Model, Store, 1>(L, a, plan_p);
    if (a.N <= 512) return launch_b<Model, Store, 2>(L, a, plan_p);
    return hipErrorInvalidValue;
  } else if constexpr (DX % 2 == 0) {
    if (a.N <= 512) return launch_b<Model, Store, 2>(L, a, plan_p);
    return hipErrorInvalidValue;
  } else {
    if (a.N <= 1024) return launch_b<Model, Store, 4>(L, a, plan_p);
    return hipErrorInvalidValue;
  }
}

template <typename Store>
static hipError_t dispatch_bm(const FwdLaunch& L, const BwdArgs& a, int* plan_p) {
  switch (L.kind) {
    case 0: return dispatch_b<LG1, Store>(L, a, plan_p);
    case 1: return dispatch_b<SV, Store>(L, a, plan_p);
    case 2:
      switch (L.dx) {
        case 2: return dispatch_b<LGD<2>, Store>(L, a, plan_p);
        case 3: return dispatch_b<LGD<3>, Store>(L, a, plan_p);
        case 4: return dispatch_b<LGD<4>, Store>(L, a, plan_p);
        case 8: return dispatch_b<LGD<8>, Store>(L, a, plan_p);
      }
  }
  return hipErrorInvalidValue;
}

// ------------------------------------------------------------ batched launches

int backward_ppt(int kind, int dx, int n) {
  const int DX = kind == 2 ? dx : 1;
  if (DX % 4 == 0) return n <= 256 ? 1 : (n <= 512 ? 2 : 0);
  if (DX % 2 == 0) return n <= 512 ? 2 : 0;
  return n <= 1024 ? 4 : 0;
}

size_t backward_smem(int fp64, int ppt, int dx) { return bwd_smem_bytes(fp64 ? 8 : 4, ppt, dx); }

template <class Model, typename Store, int PPT>
static hipError_t batch_bwd_t(const BatchLaunch& L, int* cap) {
  const void* kern;
  if constexpr (Model::DX <= 2 || Model::DX == 4) kern = reinterpret_cast<const void*>(backward_batch_kernel<Model, Store, PPT>);
  else kern = reinterpret_cast<const void*>(backward_batch_kernel_wide<Model, Store, PPT>);
  if (cap) {
    int per_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, kBlock, L.smem);
    *cap = per_cu * L.num_cus;
    return e;
  }
  const void* probs = L.probs;
  const int2* bmap = L.bmap;
  void* args[] = {&probs, &bmap};
  return hipLaunchCooperativeKernel(kern, dim3(L.blocks), dim3(kBlock), args, static_cast<unsigned>(L.smem), L.stream);
}

template <class Model, typename Store>
static hipError_t batch_bwd_ppt(const BatchLaunch& L, int* cap) {
  switch (backward_ppt(L.kind, L.dx, L.n_max)) {
    case 1: if constexpr (Model::DX % 4 == 0) return batch_bwd_t<Model, Store, 1>(L, cap); break;
    case 2: if constexpr (Model::DX % 2 == 0) return batch_bwd_t<Model, Store, 2>(L, cap); break;
    case 4: if constexpr (Model::DX % 4 != 0 && Model::DX % 2 != 0) return batch_bwd_t<Model, Store, 4>(L, cap); break;
  }
  return hipErrorInvalidValue;
}

template <typename Store>
static hipError_t batch_bwd_model(const BatchLaunch& L, int* cap) {
  switch (L.kind) {
    case 0: return batch_bwd_ppt<LG1, Store>(L, cap);
    case 1: return batch_bwd_ppt<SV, Store>(L, cap);
    case 2:
      switch (L.dx) {
        case 2: return batch_bwd_ppt<LGD<2>, Store>(L, cap);
        case 3: return batch_bwd_ppt<LGD<3>, Store>(L, cap);
        case 4: return batch_bwd_ppt<LGD<4>, Store>(L, cap);
        case 8: return batch_bwd_ppt<LGD<8>, Store>(L, cap);
      }
  }
  return hipErrorInvalidValue;
}

hipError_t backward_batch_capacity(const BatchLaunch& L, int* blocks) {
  return L.fp64 ? batch_bwd_model<double>(L, blocks) : batch_bwd_model<float>(L, blocks);
}

hipError_t launch_backward_batch(const BatchLaunch& L) {
  return L.fp64 ? batch_bwd_model<double>(L, nullptr) : batch_bwd_model<float>(L, nullptr);
}

hipError_t launch_island_grad_sum(const double* gisl, int m, int P, double* out, hipStream_t st) {
  island_grad_sum_kernel<<<dim3(1), dim3(kBlock), 0, st>>>(gisl, m, P, out);
  return hipGetLastError();
}

hipError_t launch_backward(const FwdLaunch& L, const BwdArgs& a, int* max_blocks_out) {
  return L.fp64 ? dispatch_bm<double>(L, a, max_blocks_out) : dispatch_bm<float>(L, a, max_blocks_out);
}

}  // namespace airpf
