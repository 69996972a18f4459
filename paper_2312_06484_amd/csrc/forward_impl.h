// AIRPF forward pass on gfx950: one persistent cooperative launch runs all T
// filter steps of Algorithm 1 (Heine, arXiv:2312.06484, Section 2).
//
// Work decomposition
//   * A team of TP lanes (power of two, <= 256) owns one island; lane l holds
//     particles [l*PPT, (l+1)*PPT) of it in registers, PPT >= 4 normals' worth
//     so that one Philox call feeds whole Box-Muller pairs.
//   * Block b (256 lanes) owns the c = m/G consecutive islands
//     [b*c, (b+1)*c) and processes them tpb = 256/TP at a time.
//   * Per step the only grid-wide dependency is the island-weight cascade
//     (the ENF test and the pair selections): one grid barrier per step.
//
// Step n, per island k (Algorithm 1 in order):
//   mutation     x_n = K(block pi_{n-1}(k) of step n-1's resampled state)
//                (or x_0 ~ pi_0), normals at (step n, island k);
//   weighting    lw = log g_n(x) per particle, q = floor(2^40 exp(lw - max)),
//                Q = sum q (exact), L_k = Lpre_k + ((max + log Q) + cst);
//                the particle arithmetic (normals, model, lw, exp) is done in
//                the state's precision Store, island weights in double;
//   resampling   systematic on the integer cumulative weights: slot j takes
//                min{i : N C_i > U + j Q}, U uniform on [0, Q);
//   island tree  pair means log((W_a + W_b)/2) of aligned blocks, level by
//                level (the normaliser line of Algorithm 1 applied to a
//                block's two halves); published with one ENF record
//                (E, a, b) per level (a = sum W 2^-E, b = sum W^2 2^-2E).
// After the barrier every block evaluates the ENF of each stage from the
// published records, s* = the number of leading stages with ENF < tau, and
// walks each of its islands down the stages s*, ..., 1: at stage s island
// cur takes its partner cur ^ 2^(s-1) with probability
// W_p / (W_cur + W_p) (draw at (step, island cur, stage s)).  The island's
// next weight is its 2^{s*}-block mean.  With r-ary interactions (r = 2^rb)
// stage t reads tree level (t-1) rb + 1, and the walk's island takes the
// member d of its r-group with probability W_d / sum W.
//
// ENF at stage s (W the weights after s-1 interacting stages, B_b the sums of
// the aligned 2^{s-1}-blocks): every island holds its block mean, so
// sum_k W_k = sum_b B_b and sum_k W_k^2 = 2^{s-1} sum_b (B_b / 2^{s-1})^2, and
// ENF_s = (m^-1 sum W)^2 / (m^-1 sum W^2) follows from the record of the
// level-s tree values (the block means B_b / 2^{s-1}).
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_cooperative_groups.h>
#include <stdint.h>
#include <cstdlib>
#include <type_traits>

#include "dev_models.h"
#include "dev_sync.h"
#include "internal.h"

namespace airpf {

// ------------------------------------------------------------ the kernel

// Noise values one particle consumes per step: its normals (one per state
// coordinate), or the raw words of a word-driven model.
template <class Model>
__host__ __device__ constexpr int noise_per_particle() {
  if constexpr (Model::kWordNoise) return Model::kWords; else return Model::DX;
}

// The mutation noise of one lane's particles j0 .. j0 + PPT - 1 at (step n,
// island k): PPT * DX normal variates from the lane's blocks of four, or,
// for a model driven by raw words, the first kWords words of particle j's
// own Philox blocks (counters j * B .. j * B + B - 1, B = ceil(kWords / 4),
// the model's tag), exact in double.
template <class Model, typename Store, int PPT>
__device__ __forceinline__ void draw_noise(const Key& key, int64_t n, int k, int j0, Store* z) {
  constexpr int NZ = PPT * Model::DX;
  if constexpr (Model::kWordNoise) {
    static_assert(std::is_same<Store, double>::value, "raw words are kept exactly in double");
    constexpr int W = Model::kWords, B = (W + 3) / 4;
#pragma unroll
    for (int r = 0; r < PPT; ++r) {
#pragma unroll
      for (int b = 0; b < B; ++b) {
        uint32_t w[4];
        draw4(key, static_cast<uint32_t>((j0 + r) * B + b), static_cast<uint32_t>(k), static_cast<uint32_t>(n),
              Model::kTag, 0, w);
#pragma unroll
        for (int i = 0; i < 4; ++i)
          if (4 * b + i < W) z[r * W + 4 * b + i] = static_cast<Store>(w[i]);
      }
    }
  } else {
    for (int g = 0; g < NZ / 4; ++g) {
      Store t[4];
      normals4(key, static_cast<uint32_t>((j0 * Model::DX) / 4 + g), static_cast<uint32_t>(k), static_cast<uint32_t>(n), t);
#pragma unroll
      for (int r = 0; r < 4; ++r) z[4 * g + r] = t[r];
    }
  }
}

// One problem's filter, run by the G blocks of its sub-grid; `bid` is this
// block's index within them.
// Plain: a run with no traces, no score records, no replay and no
// checkpoints, compiled on its own so that none of those paths (nor the
// registers they hold) exist in it.
// Mult: multinomial internal resampling (a kernel of its own, so that the
// systematic kernels carry none of its code or registers).
// Adapt: adaptive internal resampling (systematic when an island resamples;
// a kernel of its own, states in double, sources always from HBM).
template <class Model, typename Store, int PPT, bool Plain, bool Mult = false, bool Adapt = false>
__device__ __forceinline__ void forward_body(const FwdArgs& a, const int bid) {
  constexpr int DX = Model::DX;
  constexpr int NZ = PPT * DX;                 // normals per lane per step
  constexpr int NW = noise_per_particle<Model>(), NZW = PPT * NW;   // noise values per particle, per lane
  static_assert(NZ % 4 == 0, "a lane consumes whole Philox blocks");
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double red_d[kWaves];
  __shared__ uint64_t red_u[kWaves];
  __shared__ uint64_t bc_u[kBlock];
  __shared__ int bc_i[kWaves];
  __shared__ int s_sstar;
  __shared__ double s_enf[kWaves], s_encmax[kWaves];
  __shared__ int s_src[kMaxIslandsPerBlock];          // this step's source island of each island
  __shared__ double s_lpre[kMaxIslandsPerBlock];      // and its entering log-weight

  const int tid = threadIdx.x;
  const int TP = a.TP, tpb = kBlock / TP;
  const int team = tid / TP, lane = tid & (TP - 1);
  const int wave = tid >> 6, lane64 = tid & 63;
  const int m = a.m, N = a.N, S = a.S, c = a.c, lc = a.lc, G = a.G;
  const int rb = a.arity_log2 > 1 ? a.arity_log2 : 1, Sr = S / rb;   // r-ary interactions: Sr stages
  const int kbase = bid * c;
  const Key key = make_key(a.seed);
  const int passes = (c + tpb - 1) / tpb;
  int32_t* const tr_sstar = Plain ? nullptr : a.tr_sstar;
  double* const tr_enf = Plain ? nullptr : a.tr_enf;
  double* const tr_lpost = Plain ? nullptr : a.tr_lpost;
  int32_t* const tr_anc = Plain ? nullptr : a.tr_anc;
  int32_t* const tr_pi = Plain ? nullptr : a.tr_pi;
  unsigned long long* const tr_digest = Plain ? nullptr : a.tr_digest;
  double* const tr_fmean = Plain ? nullptr : a.tr_fmean;
  double* const tr_lpre = Plain ? nullptr : a.tr_lpre;
  void* const rec_x = Plain ? nullptr : a.rec_x;
  uint16_t* const rec_anc = Plain ? nullptr : a.rec_anc;
  void* const ck_x = Plain ? nullptr : a.ck_x;
  double* const ck_L = Plain ? nullptr : a.ck_L;
  const int64_t ck_every = Plain ? 0 : a.ck_every;
  const int ck_in = Plain ? 0 : a.ck_in;
  const int64_t n0 = Plain ? 0 : a.n0, n1 = Plain ? a.T : a.n1;

  Store* sx = reinterpret_cast<Store*>(smem);                                    // [kBlock*NZ]
  int* sA = reinterpret_cast<int*>(smem + ((sizeof(Store) * kBlock * NZ + 15) & ~size_t(15)));   // [kBlock*PPT]
  double* lvb = reinterpret_cast<double*>(sA + kBlock * PPT);                      // [2][2c]
  double* up = lvb + 4 * c;                                                       // [2G]
  // with res_lds: this block's resampled states of the last two steps, by
  // step parity, island-major as in HBM ([2][c*N*DX])
  Store* res = reinterpret_cast<Store*>(up + 2 * G);
  const int64_t res_words = static_cast<int64_t>(c) * N * DX;
  // this block's part of the island tree (levels 1 .. lc+1, level l at
  // offset 2c - 2c/2^(l-1)), one copy per step parity: the walk of step n
  // reads step n-1's copy while the weighting writes step n's
  // multinomial resampling: each team's inclusive cumulative weights
  // ([kBlock*PPT] uint64), after the resampled states when those are in LDS
  uint64_t* sC = reinterpret_cast<uint64_t*>(
      (reinterpret_cast<uintptr_t>(a.res_lds ? res + 2 * res_words : res) + 15) & ~static_cast<uintptr_t>(15));
  auto lvp = [&](int par) { return lvb + 2 * c * par; };

  unsigned epoch = 0;
  // tau so small that no stage can ever interact, and nothing traced or
  // recorded: the blocks are independent until the final log Zhat
  const bool never = a.no_interaction && !tr_enf && !tr_sstar && !tr_pi && !tr_lpost && !tr_anc &&
                     !tr_digest && !tr_fmean && !tr_lpre && !rec_x && !rec_anc && !ck_x && !ck_in;

  // levels lc+1 .. `level` of the island tree in `up`, built on demand from
  // the G published block roots (identical in every block); up_top is the
  // highest level built for the current cascade
  int up_top = 0;
  auto build_upper_to = [&](int par, int level) {
    if (up_top < lc + 1) {
      for (int b = tid; b < G; b += kBlock) up[b] = get(a.tree[par] + tree_off(m, lc + 1) + b);
      __syncthreads();
      up_top = lc + 1;
    }
    for (; up_top < level; ++up_top) {
      const int u = up_top + 1 - (lc + 1);
      const int cnt = G >> u;
      const int o_prev = 2 * G - ((2 * G) >> (u - 1)), o = 2 * G - ((2 * G) >> u);
      for (int i = tid; i < cnt; i += kBlock) up[o + i] = pair_mean(up[o_prev + 2 * i], up[o_prev + 2 * i + 1]);
      __syncthreads();
    }
  };

  // tree value, level >= 1: this block's own nodes from LDS, the block roots
  // (level lc+1) from `up` (loaded whenever a walk reaches that level), lower
  // nodes of other blocks from their published copy
  auto lt_value = [&](int par, int level, int idx) -> double {
    if (level <= lc + 1) {
      const int lo = kbase >> (level - 1);
      if (idx >= lo && idx < lo + (c >> (level - 1))) return lvp(par)[2 * c - ((2 * c) >> (level - 1)) + (idx - lo)];
      if (level == lc + 1) return up[idx];
      return get(a.tree[par] + tree_off(m, level) + idx);
    }
    const int u = level - (lc + 1);
    return up[2 * G - ((2 * G) >> u) + idx];
  };

  const bool replay = !Plain && a.replay_pi != 0;
  // normals of (step, island, particle) for this lane's particles
  auto draw_normals = [&](int64_t n, int k, int j0, Store* z) { draw_noise<Model, Store, PPT>(key, n, k, j0, z); };
  // Speculation: the stages of most steps do not interact (s* = 0), and then
  // every island continues from its own resampled block with its own weight,
  // all of which this block holds.  With the resampled states resident in
  // LDS, a block runs step n's passes under that assumption right after
  // publishing step n-1, while the other blocks arrive; the cascade then
  // confirms s* = 0 (the speculative results are kept and the resampled
  // blocks written out) or the step is run again as usual.  The results are
  // the same either way.
  const bool spec_on = a.res_lds && !never && !replay && !a.shortcut_all && !tr_enf && !tr_sstar && !tr_pi &&
                       !tr_lpost && !tr_anc && !tr_digest && !tr_fmean && !tr_lpre && !rec_x && !rec_anc && !ck_x &&
                       !ck_in;
  bool pending = false;     // step n-1 is published and its cascade not yet taken
  bool spec_done = false;   // step n's passes have run speculatively
  int64_t n = n0;
  while (n < n1) {
    const int par = static_cast<int>(n & 1), ppar = par ^ 1;
    const bool spec = spec_on && pending && !spec_done;
    // the first pass's draws (its normals and the systematic offset's first
    // block) do not depend on the other blocks: they are taken between
    // publishing this block's flag and waiting for the others
    Store z_first[NZW];
    uint32_t wsys_first[4] = {0u, 0u, 0u, 0u};
    bool first_drawn = false;
    bool skip_passes = false;
    if (pending && !spec) {
      if (!spec_done) {
        const int k0 = kbase + (team < c ? team : 0);
        draw_normals(n, k0, lane * PPT, z_first);
        if (n < a.T - 1 && lane == 0) draw4(key, 0, static_cast<uint32_t>(k0), static_cast<uint32_t>(n), kTagSys, 0, wsys_first);
        first_drawn = true;
      }
      if (!grid_wait(a.bar, G, epoch, a.status)) return;
      pending = false;
    }
    if (n > n0 && !replay && !never && !spec) {
      // ---- cascade of step n-1 (every block, identical) ----
      up_top = 0;
      int sstar = 0;
      if (a.shortcut_all) {
        // tau > 1: every stage interacts (ENF <= 1 always)
        build_upper_to(ppar, S + 1);
        if (up[2 * G - 2] == ninf()) {                               // every island dead
          if (bid == 0 && tid == 0) *a.out_logz = ninf();
          return;
        }
        sstar = Sr;
      } else {
        // ENF of up to four stages at once, one per wave; a stage that does not
        // interact leaves every weight unchanged, so every later stage sees the
        // same ENF and does not interact either (traced as that same value).
        // The first batch stops at the stages the published block records
        // cover, so a step whose first stage does not interact never needs
        // the upper tree.
        bool stop = false;
        // stage t reads tree level lev(t) = (t-1) rb + 1 (level t for pairs)
        auto lev = [&](int t) { return (t - 1) * rb + 1; };
        int s_hi = lc / rb + 1 < kWaves ? lc / rb + 1 : kWaves;
        if (s_hi > Sr) s_hi = Sr;
        for (int s0 = 1; s0 <= Sr && !stop; s0 = s_hi + 1, s_hi = s0 + kWaves - 1 < Sr ? s0 + kWaves - 1 : Sr) {
          if (lev(s_hi) > lc + 1) build_upper_to(ppar, lev(s_hi));
          const int sw = s0 + wave;
          if (sw <= s_hi) {
            const int lv = lev(sw);
            EnfRec r;
            if (lv <= lc + 1) {
              const double* ps = a.part[ppar] + static_cast<int64_t>(lv - 1) * 3 * G;
              r = wave_reduce_enf(G, [&](int i) { return EnfRec{get(ps + i), get(ps + G + i), get(ps + 2 * G + i)}; });
            } else {
              const double* lvl = up + 2 * G - ((2 * G) >> (lv - lc - 1));
              r = wave_reduce_enf(G >> (lv - lc - 1), [&](int i) { return enf_leaf(lvl[i]); });
            }
            // after the interacting stages below, every island holds the mean
            // of its aligned 2^{lv-1}-block: sum_k W_k = 2^{lv-1} sum_b w_b,
            // sum_k W_k^2 = 2^{lv-1} sum_b w_b^2
            const double blk = static_cast<double>(1 << (lv - 1));
            const double am = (blk * r.a) * __builtin_ldexp(1.0, -S), bm = (blk * r.b) * __builtin_ldexp(1.0, -S);   // m = 2^S: scaling by the exact reciprocal is the division
            if ((tid & 63) == 0) { s_enf[wave] = (am * am) / bm; s_encmax[wave] = r.E; }
          }
          __syncthreads();
          if (s0 == 1 && s_encmax[0] == ninf()) {                    // every island dead
            if (bid == 0 && tid == 0) *a.out_logz = ninf();
            return;
          }
          for (int t = s0; t <= s_hi; ++t) {
            const double enf = s_enf[t - s0];
            const bool go = enf < a.tau;
            if (tr_enf && bid == 0 && tid == 0)
              for (int q = t; q <= (go ? t : Sr); ++q) tr_enf[(n - 1) * (S + 1) + q] = enf;
            if (!go) { stop = true; break; }
            sstar = t;
          }
          __syncthreads();
        }
        if (sstar * rb + 1 > lc + 1) build_upper_to(ppar, sstar * rb + 1);
      }
      if (bid == 0 && tid == 0) {
        if (tr_sstar) tr_sstar[n - 1] = sstar;
        if (tr_digest) atomicAdd(&tr_digest[2 * (n - 1) + 1], (unsigned long long)sstar * 0x9E3779B97F4A7C15ULL);
      }
      s_sstar = sstar;
      __syncthreads();
      if (spec_done) {
        spec_done = false;
        if (sstar == 0) {
          // speculation confirmed: write the resampled blocks out
          if (n < a.T - 1) {
            Store* xo_blk = static_cast<Store*>(a.x1[par]) + static_cast<int64_t>(kbase) * N * DX;
            for (int64_t w = tid; w < res_words; w += kBlock) put(xo_blk + w, res[par * res_words + w]);
          }
          skip_passes = true;
        }
      }
    }
    const int sstar = (n > n0 && !replay && !never && !spec) ? s_sstar : 0;

    // ---- the source block and entering weight of every island of the block,
    // all islands at once: island k walks the interacting stages s*, ..., 1;
    // at stage s the island `cur` it has reached takes its partner
    // cur ^ 2^(s-1) with probability W_p / (W_cur + W_p) (its own draw at
    // (step, cur, stage s)), which composes the per-stage selections that
    // Algorithm 1 applies to every island.  Its entering weight is its
    // 2^{s*}-block mean.
    const bool mutate = n != 0 && !(n == n0 && ck_in);
    if (!skip_passes) {
    if (mutate && !spec) {
      for (int li = tid; li < c; li += kBlock) {
        const int k = kbase + li;
        int cur = k;
        double lpre = 0.0;
        if (replay) {
          cur = tr_pi[(n - 1) * m + k];
        } else {
          if (rb == 1) {
          for (int s = sstar; s >= 1; --s) {
            const int pr = cur ^ (1 << (s - 1));
            const double lc_ = lt_value(ppar, s, cur >> (s - 1));
            const double lp_ = lt_value(ppar, s, pr >> (s - 1));
            uint32_t w[4];
            draw4(key, static_cast<uint32_t>(s), static_cast<uint32_t>(cur), static_cast<uint32_t>(n - 1), kTagIsl, 0, w);
            if (uniform53(w[0], w[1]) < take_partner_prob(lc_, lp_)) cur = pr;
          }
          } else {
            // r-ary: at stage s island cur takes member d of its group (the
            // islands differing from it only in base-r digit s-1) with
            // probability W_d / sum W: the first d whose running sum of
            // exp(L_d - max L) exceeds u times the total (the last live
            // member if rounding leaves none; all dead: itself)
            const int ar = 1 << rb;
            for (int s = sstar; s >= 1; --s) {
              const int p = (s - 1) * rb;
              const int own = (cur >> p) & (ar - 1);
              const int b0 = (cur >> p) - own;               // the group's first member at level p + 1
              uint32_t w[4];
              draw4(key, static_cast<uint32_t>(s), static_cast<uint32_t>(cur), static_cast<uint32_t>(n - 1), kTagIsl, 0, w);
              const double u = uniform53(w[0], w[1]);
              double hi = ninf();
              for (int d = 0; d < ar; ++d) {
                const double v = lt_value(ppar, p + 1, b0 + d);
                hi = v > hi ? v : hi;
              }
              int pick = own;
              if (hi != ninf()) {
                double tot = 0.0;
                for (int d = 0; d < ar; ++d) tot += dexp(lt_value(ppar, p + 1, b0 + d) - hi);
                const double t = u * tot;
                double run = 0.0;
                int last = own;
                bool found = false;
                for (int d = 0; d < ar && !found; ++d) {
                  const double wd = dexp(lt_value(ppar, p + 1, b0 + d) - hi);
                  run += wd;
                  if (wd > 0.0) last = d;
                  if (t < run) { pick = d; found = true; }
                }
                if (!found) pick = last;
              }
              cur = (b0 + pick) << p | (cur & ((1 << p) - 1));
            }
          }
          lpre = lt_value(ppar, sstar * rb + 1, k >> (sstar * rb));
          if (tr_pi) tr_pi[(n - 1) * m + k] = cur;
          if (tr_digest) atomicAdd(&tr_digest[2 * (n - 1) + 1], digest_term(n - 1, k, 4095, cur));
        }
        s_src[li] = cur;
        s_lpre[li] = lpre;
      }
      __syncthreads();
    }

    for (int p = 0; p < passes; ++p) {
      const int li = p * tpb + team;
      const bool active = li < c;
      const int k = kbase + (active ? li : 0);
      const int j0 = lane * PPT;

      // ---- mutation (or initial draw) ----
      const bool pre = first_drawn && p == 0;
      // sub-block 0 of the systematic offset's draw (it does not depend on Q)
      uint32_t wsys[4] = {wsys_first[0], wsys_first[1], wsys_first[2], wsys_first[3]};
      if (!pre && n < a.T - 1 && lane == 0) draw4(key, 0, static_cast<uint32_t>(k), static_cast<uint32_t>(n), kTagSys, 0, wsys);
      Store x[PPT][DX];
      double Lpre = 0.0;
      double lcr[PPT];                        // Adapt: the particles' carried log-weights
      double dqs = 0.0;                       // and the island's carried log normaliser
#pragma unroll
      for (int r = 0; r < PPT; ++r) lcr[r] = 0.0;
      if (n == n0 && ck_in) {
        // restart from the checkpoint taken entering this step
        const Store* xc = static_cast<const Store*>(ck_x) + (n / ck_every) * (static_cast<int64_t>(m) * N * DX) +
                          static_cast<int64_t>(k) * N * DX;
#pragma unroll
        for (int r = 0; r < PPT; ++r)
#pragma unroll
          for (int d = 0; d < DX; ++d) x[r][d] = (j0 + r < N) ? xc[(j0 + r) * DX + d] : Store(0);
        if (lane == 0) Lpre = ck_L[(n / ck_every) * m + k];
      } else if (n == 0) {
        Store z[NZW];
        draw_normals(n, k, j0, z);
#pragma unroll
        for (int r = 0; r < PPT; ++r) Model::template init<Store>(a.mp, z + r * NW, x[r]);
      } else {
        const int src = spec ? k : s_src[active ? li : 0];
        if (lane == 0 && active) Lpre = spec ? lvp(ppar)[li] : s_lpre[li];
        if constexpr (Adapt) {
          const double* lin = a.lc1[ppar] + static_cast<int64_t>(src) * N;
#pragma unroll
          for (int r = 0; r < PPT; ++r) lcr[r] = (j0 + r < N) ? get(lin + j0 + r) : 0.0;
          if (lane == 0 && active) dqs = get(a.dq1[ppar] + src);
        }
        // the source block's loads go out first; the normals do not need them.
        // A source island of this block is read from its LDS copy.
        Store xr[PPT][DX];
        if (a.res_lds && src >= kbase && src < kbase + c) {
          const Store* xin = res + ppar * res_words + static_cast<int64_t>(src - kbase) * N * DX;
#pragma unroll
          for (int r = 0; r < PPT; ++r)
#pragma unroll
            for (int d = 0; d < DX; ++d) xr[r][d] = (j0 + r < N) ? xin[(j0 + r) * DX + d] : Store(0);
        } else {
          const Store* xin = static_cast<const Store*>(a.x1[ppar]) + (static_cast<int64_t>(src) * N) * DX;
#pragma unroll
          for (int r = 0; r < PPT; ++r)
#pragma unroll
            for (int d = 0; d < DX; ++d) xr[r][d] = (j0 + r < N) ? get(xin + (j0 + r) * DX + d) : Store(0);
        }
        Store z[NZW];
        if (pre) {
#pragma unroll
          for (int i = 0; i < NZW; ++i) z[i] = z_first[i];
        } else {
          draw_normals(n, k, j0, z);
        }
#pragma unroll
        for (int r = 0; r < PPT; ++r) {
          Store xp[DX];
#pragma unroll
          for (int d = 0; d < DX; ++d) xp[d] = xr[r][d];
          Model::template prop<Store>(a.mp, xp, z + r * NW, x[r]);
        }
      }

      // ---- what the score records: the state entering this weighting ----
      if (active) {
        if (rec_x) {
          Store* rx = static_cast<Store*>(rec_x) + ((n - n0) * m + k) * static_cast<int64_t>(N) * DX;
#pragma unroll
          for (int r = 0; r < PPT; ++r)
#pragma unroll
            for (int d = 0; d < DX; ++d)
              if (j0 + r < N) rx[(j0 + r) * DX + d] = static_cast<Store>(x[r][d]);
        }
        if (ck_every > 0 && n % ck_every == 0 && !replay && ck_x) {
          Store* xc = static_cast<Store*>(ck_x) + (n / ck_every) * (static_cast<int64_t>(m) * N * DX) +
                      static_cast<int64_t>(k) * N * DX;
#pragma unroll
          for (int r = 0; r < PPT; ++r)
#pragma unroll
            for (int d = 0; d < DX; ++d)
              if (j0 + r < N) xc[(j0 + r) * DX + d] = static_cast<Store>(x[r][d]);
          if (lane == 0) ck_L[(n / ck_every) * m + k] = Lpre;
        }
        if (lane == 0 && tr_lpre && !replay) tr_lpre[n * m + k] = Lpre;
      }

      // ---- weighting ----
      const double* yn = a.y + n * a.dy;
      if (a.check_y && lane == 0 && active) {           // observations the host could not check
        bool fin = true;
        for (int i = 0; i < a.dy; ++i) fin = fin && isfinite(yn[i]);
        if (!fin) put(a.bad_y, 1);
      }
      Store lw[PPT];
      Store mx = neg_inf<Store>();
#pragma unroll
      for (int r = 0; r < PPT; ++r) {
        const bool valid = active && (j0 + r < N);
        Store v = valid ? Model::template logpot<Store>(a.mp, x[r], yn) : neg_inf<Store>();
        if (!(v == v)) v = neg_inf<Store>();
        if constexpr (Adapt) v = static_cast<Store>(lcr[r]) + v;     // the weight carried in
        lw[r] = v;
        mx = rmax(mx, v);
      }
      mx = team_max(mx, TP, red_d);
      uint64_t q[PPT];
      uint64_t tsum = 0;
#pragma unroll
      for (int r = 0; r < PPT; ++r) {
        q[r] = (mx == neg_inf<Store>()) ? 0 : static_cast<uint64_t>(rexp(lw[r] - mx) * Store(0x1p40));
        tsum += q[r];
      }
      const uint64_t incl = team_scan_u64(tsum, TP, red_u);
      // Q = sum_i q_i of the island: the scan's value in the team's last lane
      const uint64_t Qk = TP == 64 ? readlane_u64(incl, 63)
                          : (TP < 64 ? __shfl(incl, (tid & 63) | (TP - 1), 64) : team_sum_u64(tsum, TP, red_u));
      if (lane == 0 && active && !replay) {
        double L = (Qk == 0) ? ninf() : Lpre + ((static_cast<double>(mx) + dlog(static_cast<double>(Qk))) + a.cst_q);
        if constexpr (Adapt) {
          if (Qk != 0) L = L - dqs;                        // the incoming weights' normaliser
        }
        lvp(par)[li] = L;
        if (tr_lpost) tr_lpost[n * m + k] = L;
      }
      // Adapt: whether the island resamples, from the ESS of its weights
      // truncated to their top 20 of 40 bits (exact integer sums)
      bool resamp = true;
      if constexpr (Adapt) {
        uint64_t t1 = 0, t2 = 0;
#pragma unroll
        for (int r = 0; r < PPT; ++r) {
          const uint64_t qt = q[r] >> 20;
          t1 += qt;
          t2 += qt * qt;
        }
        const uint64_t Qt = team_sum_u64(t1, TP, red_u), S2 = team_sum_u64(t2, TP, red_u);
        resamp = Qk != 0 && S2 != 0 &&
                 static_cast<double>(Qt) * static_cast<double>(Qt) < a.ess_frac * static_cast<double>(N) * static_cast<double>(S2);
      }
      if (tr_fmean) {
        // the island's estimate of the filtering mean of x[0]: sum_i q_i x_i / Q
        double num = 0.0;
#pragma unroll
        for (int r = 0; r < PPT; ++r) num += (active && j0 + r < N) ? static_cast<double>(q[r]) * static_cast<double>(x[r][0]) : 0.0;
        num = team_sum_f64(num, TP, red_d);
        if (lane == 0 && active) tr_fmean[n * m + k] = Qk == 0 ? __longlong_as_double(0x7ff8000000000000LL) : num / static_cast<double>(Qk);
      }

      // ---- internal resampling ----
      if (n < a.T - 1) {
        Store* sxt = sx + team * TP * NZ;
        int* sAt = sA + team * TP * PPT;
#pragma unroll
        for (int r = 0; r < PPT; ++r) {
#pragma unroll
          for (int d = 0; d < DX; ++d) sxt[(j0 + r) * DX + d] = static_cast<Store>(x[r][d]);
          sAt[j0 + r] = -1;                                   // no run starts here (yet)
        }
        if constexpr (Mult) {
          // N independent draws from the island's weighted particles: slot j
          // takes the first particle whose cumulative weight exceeds U_j,
          // U_j uniform on [0, Q) (its own draw at (slot j, island, step))
          uint64_t* sCt = sC + team * TP * PPT;
          uint64_t Cr = incl - tsum;
#pragma unroll
          for (int r = 0; r < PPT; ++r) {
            Cr += q[r];
            sCt[j0 + r] = Cr;
          }
          team_sync(TP);
          // one slot at a time (not unrolled): the draws would otherwise hold
          // registers the rest of the kernel needs
#pragma unroll 1
          for (int r = 0; r < PPT; ++r) {
            const int j = j0 + r;
            if (active && j < N) {
              int anc = j;
              if (Qk > 0) {
                const uint64_t Uj = bounded_u64(key, static_cast<uint32_t>(j), static_cast<uint32_t>(k),
                                                static_cast<uint32_t>(n), kTagMult, Qk);
                int lo = 0, hi = N - 1;
                while (lo < hi) {
                  const int mid = (lo + hi) >> 1;
                  if (sCt[mid] > Uj) hi = mid; else lo = mid + 1;
                }
                anc = lo;
              }
              sAt[j] = anc;
            }
          }
        } else {
        uint64_t U = 0;
        if (lane == 0 && active && Qk > 0)
          U = bounded_u64_from(wsys, key, 0, static_cast<uint32_t>(k), static_cast<uint32_t>(n), kTagSys, Qk);
        U = team_bcast(U, TP, bc_u);
        // Slot j takes min{i : N C_i > U + j Q}.  Equivalently particle i owns
        // the slots [S(C_{i-1}), S(C_i)) with S(C) = #{j < N : U + j Q < N C}
        // = 0 if N C <= U, else min(N, floor((N C - U - 1) / Q) + 1): each
        // particle marks the first slot of its run, and a slot's ancestor is
        // the last mark at or before it.  The quotient is estimated in double
        // precision (within one of the exact one, as x / Q < N <= 2048, so
        // 32 bits hold it) and corrected in integers.
        const double rQ = 1.0 / static_cast<double>(Qk);
        auto S_of = [&](uint64_t C) -> int {
          const uint64_t NC = static_cast<uint64_t>(N) * C;
          const uint64_t xq = NC > U ? NC - U - 1 : 0;
          uint32_t qd = static_cast<uint32_t>(static_cast<double>(xq) * rQ);
          uint64_t pr = static_cast<uint64_t>(qd) * Qk;
          if (pr > xq) { qd -= 1u; pr -= Qk; }
          if (xq - pr >= Qk) qd += 1u;
          const uint32_t sv = qd + 1u;
          return NC <= U ? 0 : (sv < static_cast<uint32_t>(N) ? static_cast<int>(sv) : N);
        };
        // S at the lane's prefix sums; S of the sum before its first
        // particle (C_{j0-1}) is its left neighbour's last, 0 at a team's
        // first lane, evaluated where the neighbour is in another wave
        const uint64_t C0 = incl - tsum;                       // C_{j0-1}
        uint64_t C = C0;
        int sc[PPT];
#pragma unroll
        for (int r = 0; r < PPT; ++r) {
          C += q[r];
          sc[r] = S_of(C);
        }
        const int left = __shfl(sc[PPT - 1], lane64 == 0 ? 0 : lane64 - 1, 64);
        int s_prev = lane == 0 ? 0 : (lane64 == 0 ? S_of(C0) : left);
        team_sync(TP);
#pragma unroll
        for (int r = 0; r < PPT; ++r) {
          if (active && Qk > 0 && j0 + r < N && sc[r] > s_prev) sAt[s_prev] = j0 + r;
          s_prev = sc[r];
        }
        team_sync(TP);
        int mk[PPT];
#pragma unroll
        for (int r = 0; r < PPT; ++r) {
          const int v = (j0 + r < N) ? sAt[j0 + r] : -1;
          mk[r] = r == 0 ? v : (v > mk[r - 1] ? v : mk[r - 1]);
        }
        const int before = team_exclusive_max(mk[PPT - 1], TP, bc_i);
#pragma unroll
        for (int r = 0; r < PPT; ++r) {
          const int j = j0 + r;
          if (active && j < N) sAt[j] = (Qk > 0 && resamp) ? (mk[r] > before ? mk[r] : before) : j;
        }
        }  // systematic
        // (each lane reads back only the ancestors of its own slots)
        Store* xo = static_cast<Store*>(a.x1[par]) + (static_cast<int64_t>(k) * N) * DX;
        unsigned long long dig = 0;
#pragma unroll
        for (int r = 0; r < PPT; ++r) {
          const int j = j0 + r;
          if (active && j < N) {
            const int anc = sAt[j];
            if (tr_anc) tr_anc[(n * m + k) * static_cast<int64_t>(N) + j] = anc;
            if (rec_anc) rec_anc[((n - n0) * m + k) * static_cast<int64_t>(N) + j] = static_cast<uint16_t>(anc);
            if (tr_digest) dig += digest_term(n, k, j, anc);
          }
        }
        if (tr_digest) {
          dig = team_sum_u64(dig, TP, red_u);
          if (lane == 0 && active) atomicAdd(&tr_digest[2 * n], dig);
        }
        team_sync(TP);
        // the resampled block, written word by word with consecutive lanes on
        // consecutive words so every store instruction covers whole lines
        if (active) {
#pragma unroll
          for (int r = 0; r < NZ; ++r) {
            const int w = r * TP + lane;
            const int j = w / DX, d = w - j * DX;
            if (j < N) {
              const Store v = sxt[sAt[j] * DX + d];
              if (!spec) put(xo + w, v);
              if (a.res_lds) res[par * res_words + static_cast<int64_t>(li) * N * DX + w] = v;
            }
          }
        }
        if constexpr (Adapt) {
          // carried into the next weighting: nothing after a resampling,
          // else each particle's log fixed-point weight and the island's
          // log Q - log N
          if (active) {
            double* lo = a.lc1[par] + static_cast<int64_t>(k) * N;
#pragma unroll
            for (int r = 0; r < PPT; ++r)
              if (j0 + r < N) put(lo + j0 + r, resamp ? 0.0 : dlog(static_cast<double>(q[r])));
            if (lane == 0) put(a.dq1[par] + k, resamp ? 0.0 : dlog(static_cast<double>(Qk)) - a.log_N);
          }
        }
        team_sync(TP);
      }
    }
    __syncthreads();
    if (spec) { spec_done = true; continue; }
    }  // !skip_passes
    if (!(replay || (never && n < a.T - 1))) {

    // ---- this block's part of the island tree and the ENF partial records ----
    double* lv = lvp(par);
    if (c <= 64) {
      // one wave: lane i holds value i of the level below
      if (wave == 0) {
        double v = (lane64 < c) ? lv[lane64] : ninf();
        for (int l = 2; l <= lc + 1; ++l) {
          const int cnt = c >> (l - 1);
          const int o = 2 * c - ((2 * c) >> (l - 1));
          const double v0 = __shfl(v, (2 * lane64) & 63, 64), v1 = __shfl(v, (2 * lane64 + 1) & 63, 64);
          const double nv = lane64 < cnt ? pair_mean(v0, v1) : ninf();
          if (lane64 < cnt) lv[o + lane64] = nv;
          v = nv;
        }
      }
    } else {
      for (int l = 2; l <= lc + 1; ++l) {
        const int cnt = c >> (l - 1);
        const int o_prev = 2 * c - ((2 * c) >> (l - 2)), o = 2 * c - ((2 * c) >> (l - 1));
        for (int i = tid; i < cnt; i += kBlock) lv[o + i] = pair_mean(lv[o_prev + 2 * i], lv[o_prev + 2 * i + 1]);
        __syncthreads();
      }
    }
    __syncthreads();
    for (int l = 1; l <= lc + 1; ++l) {
      const int cnt = c >> (l - 1);
      const int o = 2 * c - ((2 * c) >> (l - 1));
      double* dst = a.tree[par] + tree_off(m, l) + (kbase >> (l - 1));
      for (int i = tid; i < cnt; i += kBlock) put(dst + i, lv[o + i]);
    }
    // ENF record of each level's values in this block, one wave per level
    for (int l = 1 + wave; l <= lc + 1; l += kWaves) {
      const int cnt = c >> (l - 1);
      const int o = 2 * c - ((2 * c) >> (l - 1));
      const EnfRec r = wave_reduce_enf(cnt, [&](int i) { return enf_leaf(lv[o + i]); });
      if (lane64 == 0) {
        double* pl = a.part[par] + static_cast<int64_t>(l - 1) * 3 * G;
        put(pl + bid, r.E);
        put(pl + G + bid, r.a);
        put(pl + 2 * G + bid, r.b);
      }
    }
    }  // tree
    ++n;
    // a recomputed step n reads step n-1's resampled blocks through the maps
    // of s*_{n-1} and overwrites the buffer that step n-1 read through those
    // of s*_{n-2}; when neither reaches outside this block (s* <= log2 c), a
    // block barrier orders everything the step touches
    const bool local_replay = replay && a.sstar_in && a.sstar_in[n - 1] <= lc &&
                              (n < 2 || a.sstar_in[n - 2] <= lc);
    if (n < n1 && !never && !local_replay) {
      grid_arrive(a.bar, bid, epoch);
      pending = true;
    }
  }

  // ---- log Zhat after the last weighting: log of the mean island weight,
  // the root of the island tree ----
  if (replay || n1 < a.T) return;
  if (!grid_barrier(a.bar, G, bid, epoch, a.status)) return;
  if (bid == 0) {
    up_top = 0;
    build_upper_to(static_cast<int>((a.T - 1) & 1), S + 1);
    const double lroot = up[2 * G - 2];
    if (tid == 0) {
      *a.out_logz = lroot;
      if (tr_sstar) tr_sstar[a.T - 1] = 0;
    }
  }
}

// ------------------------------------------------------------ pipelined forward
// Untraced runs whose resampled states fit the block's LDS copy and whose
// teams lie inside one wave (TP <= 64), with tau <= 1 (tau <= 1/(2m): no
// stage can interact, and nothing is exchanged until the final log Zhat).
//
// Most steps do not interact, and then a block's next step needs nothing
// from the other blocks.  A block of this kernel has four worker waves
// (the island passes, exactly those of forward_body) and one control wave
// that does everything involving other blocks.  Between two joins (block
// barriers) the workers run step n on the assumption that steps n-1 and
// n-2 do not interact (every island continues from its own resampled block
// with its own weight, all in LDS), while the control wave sends out its
// level-1 ENF record of step n-1 and decides step n-2 from the records sent
// out one iteration earlier, evaluating the stages one at a time until one
// does not interact.  When step n-2 interacts, steps n-1 (from the walk's
// sources; all blocks have passed the interaction's barrier by then) and n
// are run again.  Every value is computed by the same operations as in
// forward_body, so the results are identical.
//
// Stage 1 needs only the blocks' level-1 ENF records, so the control wave
// publishes those alone (in a ring where a record is also the block's
// arrival); the island tree and the other levels' records follow (with a
// flag barrier) only when stage 1 interacts, which every block decides
// alike.  Only then can another block
// read this block's resampled states of that step (in the rerun of the next
// step), so they are copied from LDS to HBM at that point, not by the
// passes: a step whose stage 1 does not interact moves no state through
// HBM at all.
constexpr int kPipeBlock = kBlock + 64;
constexpr int kYChunk = 64;                 // observation steps per LDS chunk

// Rec: the forward run of the score, which also keeps each step's island
// maps, s*, entering weights, and checkpoints every ck_every steps (no
// other trace, no replay).
// TPC > 0: compiled for teams of TPC lanes and full islands (N = TPC * PPT),
// so that the team reductions, scans and bounds are resolved at compile
// time (no branch on the team width); 0: any width, read from the arguments.
// Rary: r-ary interactions (r = 2^arity_log2): the control wave's cascade
// and walk over the groups of r islands (untraced runs).
// Mult: multinomial internal resampling in the workers' passes (untraced
// runs), as in forward_body.
template <class Model, typename Store, int PPT, bool Rec, int TPC = 0, bool Rary = false, bool Mult = false>
__device__ __forceinline__ void forward_pipe_body(const FwdArgs& a, const int bid) {
  constexpr int DX = Model::DX;
  constexpr int NZ = PPT * DX;
  constexpr int NW = noise_per_particle<Model>(), NZW = PPT * NW;
  static_assert(NZ % 4 == 0, "a lane consumes whole Philox blocks");
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double red_d[kWaves];            // team helpers' scratch (unused for TP <= 64)
  __shared__ uint64_t red_u[kWaves];
  __shared__ uint64_t bc_u[kBlock];
  __shared__ int bc_i[kWaves];
  __shared__ int s_src[kMaxIslandsPerBlock];
  __shared__ double s_lpre[kMaxIslandsPerBlock];
  __shared__ int s_ctl[2];                    // s* of the step just decided; 1: leave
  // the observations of 64 steps at a time, two chunks: the control wave
  // loads chunk j + 1 while the workers use chunk j, so that no worker pass
  // waits on a memory load for its observation
  __shared__ double s_y[2][kYChunk * kMaxDy];
  // each island's level-1 ENF leaf (E, a, b) by step parity, formed by the
  // island's team right after its weighting (the control wave only joins
  // the block's leaves)
  __shared__ EnfRec s_leaf[3][kMaxIslandsPerBlock];

  const int tid = threadIdx.x;
  const bool ctl = tid >= kBlock;             // the control wave
  const int lane64 = tid & 63;
  const int TP = TPC ? TPC : a.TP, tpb = kBlock / TP;
  const int team = tid / TP, lane = tid & (TP - 1);
  const int m = a.m, N = TPC ? TPC * PPT : a.N, S = a.S, c = a.c, lc = a.lc, G = a.G;
  const int64_t T = a.T;
  const int kbase = bid * c;
  const Key key = make_key(a.seed);
  const int passes = (c + tpb - 1) / tpb;
  int32_t* const tr_pi = Rec ? a.tr_pi : nullptr;
  int32_t* const tr_sstar = Rec ? a.tr_sstar : nullptr;
  double* const tr_lpre = Rec ? a.tr_lpre : nullptr;
  void* const ck_x = Rec ? a.ck_x : nullptr;
  double* const ck_L = Rec ? a.ck_L : nullptr;
  const int64_t ck_every = Rec ? a.ck_every : 0;

  Store* sx = reinterpret_cast<Store*>(smem);                                    // [kBlock*NZ]
  int* sA = reinterpret_cast<int*>(smem + ((sizeof(Store) * kBlock * NZ + 15) & ~size_t(15)));   // [kBlock*PPT]
  double* lvb = reinterpret_cast<double*>(sA + kBlock * PPT);                      // [3][2c]
  double* up = lvb + 6 * c;                                                       // [2G]
  Store* res = reinterpret_cast<Store*>(up + 2 * G);                              // [3][c*N*DX]
  const int64_t res_words = static_cast<int64_t>(c) * N * DX;
  // Mult: each team's inclusive cumulative weights ([kBlock*PPT] uint64)
  [[maybe_unused]] uint64_t* sC = reinterpret_cast<uint64_t*>(
      (reinterpret_cast<uintptr_t>(res + 3 * res_words) + 15) & ~static_cast<uintptr_t>(15));
  // a step's island log-weights (and local tree) and resampled states live
  // in slot step mod 3: the steps being decided, published and run
  auto lvp = [&](int sl) { return lvb + 2 * c * sl; };
  auto wsync = [] {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  };

  // ================= worker waves: the island passes of step n =================
  // spec: sources and entering weights under s*_{n-1} = 0
  // a team with one island per step (one pass) draws the first block of
  // the systematic-resampling words of its next TP steps at once, lane l
  // the block of step base + l; the words are the same either way
  const bool sys_batch = passes == 1 && TP >= 16;
  uint32_t sysw[4] = {0u, 0u, 0u, 0u};
  int64_t sys_base = -1;                      // first step of the batch in sysw
  auto run_passes = [&](int64_t n, bool spec) {
    const int ppar = static_cast<int>((n & 1) ^ 1);                // HBM copies of step n-1, by parity
    const int n32 = static_cast<int>(n);                           // steps are below 2^30
    const int sl = n32 % 3, psl = (n32 + 2) % 3;                   // LDS slots of steps n, n-1
    // the observation of step n, loaded ahead of the mutation (the kernel
    // compiled for a team width runs the one-dimensional models, whose
    // observations are one value)
    double y_early = 0.0;
    if constexpr (TPC > 0) y_early = s_y[(n32 / kYChunk) & 1][n32 % kYChunk];
    for (int p = 0; p < passes; ++p) {
      const int li = p * tpb + team;
      const bool active = li < c;
      const int k = kbase + (active ? li : 0);
      const int j0 = lane * PPT;
      uint32_t wsys[4] = {0u, 0u, 0u, 0u};
      if (sys_batch) {
        // (a step run again may belong to the batch before the one drawn last)
        const int64_t base = n - n % TP;
        if (base != sys_base) {
          if (base + lane < T - 1)
            draw4(key, 0, static_cast<uint32_t>(k), static_cast<uint32_t>(base + lane), kTagSys, 0, sysw);
          sys_base = base;
        }
        if (TP == 64) {
          // one team per wave: the step's lane is the same for every lane
          const int sl_ = static_cast<int>(n - base);
#pragma unroll
          for (int i = 0; i < 4; ++i) wsys[i] = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(sysw[i]), sl_));
        } else {
          const int src_lane = (tid & 63 & ~(TP - 1)) | static_cast<int>(n - base);
#pragma unroll
          for (int i = 0; i < 4; ++i) wsys[i] = static_cast<uint32_t>(__shfl(static_cast<int>(sysw[i]), src_lane, 64));
        }
      } else if (n < T - 1 && lane == 0) {
        draw4(key, 0, static_cast<uint32_t>(k), static_cast<uint32_t>(n), kTagSys, 0, wsys);
      }
      Store x[PPT][DX];
      double Lpre = 0.0;
      if (n == 0) {
        Store z[NZW];
        draw_noise<Model, Store, PPT>(key, n, k, j0, z);
#pragma unroll
        for (int r = 0; r < PPT; ++r) Model::template init<Store>(a.mp, z + r * NW, x[r]);
      } else {
        const int src = spec ? k : s_src[active ? li : 0];
        if (lane == 0 && active) Lpre = spec ? lvp(psl)[li] : s_lpre[li];
        Store xr[PPT][DX];
        if (src >= kbase && src < kbase + c) {
          const Store* xin = res + psl * res_words + static_cast<int64_t>(src - kbase) * N * DX;
#pragma unroll
          for (int r = 0; r < PPT; ++r)
#pragma unroll
            for (int d = 0; d < DX; ++d) xr[r][d] = (j0 + r < N) ? xin[(j0 + r) * DX + d] : Store(0);
        } else {
          const Store* xin = static_cast<const Store*>(a.x1[ppar]) + (static_cast<int64_t>(src) * N) * DX;
#pragma unroll
          for (int r = 0; r < PPT; ++r)
#pragma unroll
            for (int d = 0; d < DX; ++d) xr[r][d] = (j0 + r < N) ? get(xin + (j0 + r) * DX + d) : Store(0);
        }
        Store z[NZW];
        draw_noise<Model, Store, PPT>(key, n, k, j0, z);
#pragma unroll
        for (int r = 0; r < PPT; ++r) {
          Store xp[DX];
#pragma unroll
          for (int d = 0; d < DX; ++d) xp[d] = xr[r][d];
          Model::template prop<Store>(a.mp, xp, z + r * NW, x[r]);
        }
      }

      // ---- what the score keeps: the entering weight, and the state
      // entering this weighting at checkpoint steps (a step run again
      // rewrites them) ----
      if (Rec && active) {
        if (ck_every > 0 && n % ck_every == 0 && ck_x) {
          Store* xc = static_cast<Store*>(ck_x) + (n / ck_every) * (static_cast<int64_t>(m) * N * DX) +
                      static_cast<int64_t>(k) * N * DX;
#pragma unroll
          for (int r = 0; r < PPT; ++r)
#pragma unroll
            for (int d = 0; d < DX; ++d)
              if (j0 + r < N) xc[(j0 + r) * DX + d] = static_cast<Store>(x[r][d]);
          if (lane == 0) ck_L[(n / ck_every) * m + k] = Lpre;
        }
        if (lane == 0 && tr_lpre) tr_lpre[n * m + k] = Lpre;
      }

      // ---- weighting ----
      const double* yn = s_y[(n32 / kYChunk) & 1] + (n32 % kYChunk) * a.dy;
      const double yreg[1] = {y_early};
      Store lw[PPT];
      Store mx = neg_inf<Store>();
#pragma unroll
      for (int r = 0; r < PPT; ++r) {
        const bool valid = active && (j0 + r < N);
        Store v = valid ? Model::template logpot<Store>(a.mp, x[r], TPC > 0 ? yreg : yn) : neg_inf<Store>();
        if (!(v == v)) v = neg_inf<Store>();
        lw[r] = v;
        mx = rmax(mx, v);
      }
      mx = team_max(mx, TP, red_d);
      uint64_t q[PPT];
      uint64_t tsum = 0;
#pragma unroll
      for (int r = 0; r < PPT; ++r) {
        q[r] = (mx == neg_inf<Store>()) ? 0 : static_cast<uint64_t>(rexp(lw[r] - mx) * Store(0x1p40));
        tsum += q[r];
      }
      const uint64_t incl = team_scan_u64(tsum, TP, red_u);
      const uint64_t Qk = TP == 64 ? readlane_u64(incl, 63) : __shfl(incl, (tid & 63) | (TP - 1), 64);
      if (lane == 0 && active) {
        const double L = (Qk == 0) ? ninf() : Lpre + ((static_cast<double>(mx) + dlog(static_cast<double>(Qk))) + a.cst_q);
        lvp(sl)[li] = L;
        s_leaf[sl][li] = enf_leaf(L);
      }

      // ---- internal resampling (systematic, by offspring counts) ----
      if (n < T - 1) {
        Store* sxt = sx + team * TP * NZ;
        int* sAt = sA + team * TP * PPT;
#pragma unroll
        for (int r = 0; r < PPT; ++r) {
#pragma unroll
          for (int d = 0; d < DX; ++d) sxt[(j0 + r) * DX + d] = static_cast<Store>(x[r][d]);
          sAt[j0 + r] = -1;
        }
        if constexpr (Mult) {
          // N independent draws: slot j takes the first particle whose
          // cumulative weight exceeds U_j, uniform on [0, Q) (its own draw at
          // (slot j, island, step)), found by binary search
          uint64_t* sCt = sC + team * TP * PPT;
          uint64_t Cr = incl - tsum;
#pragma unroll
          for (int r = 0; r < PPT; ++r) {
            Cr += q[r];
            sCt[j0 + r] = Cr;
          }
          team_sync(TP);
#pragma unroll 1
          for (int r = 0; r < PPT; ++r) {
            const int j = j0 + r;
            if (active && j < N) {
              int anc = j;
              if (Qk > 0) {
                const uint64_t Uj = bounded_u64(key, static_cast<uint32_t>(j), static_cast<uint32_t>(k),
                                                static_cast<uint32_t>(n), kTagMult, Qk);
                int lo = 0, hi = N - 1;
                while (lo < hi) {
                  const int mid = (lo + hi) >> 1;
                  if (sCt[mid] > Uj) hi = mid; else lo = mid + 1;
                }
                anc = lo;
              }
              sAt[j] = anc;
            }
          }
        } else {
        uint64_t U = 0;
        if (lane == 0 && active && Qk > 0)
          U = bounded_u64_from(wsys, key, 0, static_cast<uint32_t>(k), static_cast<uint32_t>(n), kTagSys, Qk);
        U = team_bcast(U, TP, bc_u);
        const double rQ = 1.0 / static_cast<double>(Qk);
        // x < N C <= N Q, so the quotient x / Q is below N <= 2048 and 32 bits
        // hold it (and its estimate, within one of it)
        auto S_of = [&](uint64_t C) -> int {
          const uint64_t NC = static_cast<uint64_t>(N) * C;
          const uint64_t xq = NC > U ? NC - U - 1 : 0;
          uint32_t qd = static_cast<uint32_t>(static_cast<double>(xq) * rQ);
          uint64_t pr = static_cast<uint64_t>(qd) * Qk;
          if (pr > xq) { qd -= 1u; pr -= Qk; }
          if (xq - pr >= Qk) qd += 1u;
          const uint32_t sv = qd + 1u;
          return NC <= U ? 0 : (sv < static_cast<uint32_t>(N) ? static_cast<int>(sv) : N);
        };
        // S at the lane's prefix sums; S of the sum before its first
        // particle is its left neighbour's last (0 at a team's first lane)
        uint64_t C = incl - tsum;
        int sc[PPT];
#pragma unroll
        for (int r = 0; r < PPT; ++r) {
          C += q[r];
          sc[r] = S_of(C);
        }
        const int left = __shfl(sc[PPT - 1], lane64 == 0 ? 0 : lane64 - 1, 64);
        int s_prev = lane == 0 ? 0 : left;                     // (teams lie inside one wave)
        team_sync(TP);
#pragma unroll
        for (int r = 0; r < PPT; ++r) {
          if (active && Qk > 0 && j0 + r < N && sc[r] > s_prev) sAt[s_prev] = j0 + r;
          s_prev = sc[r];
        }
        team_sync(TP);
        int mk[PPT];
#pragma unroll
        for (int r = 0; r < PPT; ++r) {
          const int v = (j0 + r < N) ? sAt[j0 + r] : -1;
          mk[r] = r == 0 ? v : (v > mk[r - 1] ? v : mk[r - 1]);
        }
        const int before = team_exclusive_max(mk[PPT - 1], TP, bc_i);
#pragma unroll
        for (int r = 0; r < PPT; ++r) {
          const int j = j0 + r;
          if (active && j < N) sAt[j] = Qk > 0 ? (mk[r] > before ? mk[r] : before) : j;
        }
        }  // systematic
        team_sync(TP);
        if (active) {
#pragma unroll
          for (int r = 0; r < NZ; ++r) {
            const int w = r * TP + lane;
            const int j = w / DX, d = w - j * DX;
            if (j < N) res[sl * res_words + static_cast<int64_t>(li) * N * DX + w] = sxt[sAt[j] * DX + d];
          }
        }
        team_sync(TP);
      }
    }
  };

  // ================= control wave =================
  unsigned epoch = 0;
  int up_top = 0;
  auto build_upper_to = [&](int64_t t, int level) {
    const int par = static_cast<int>(t & 1);
    if (up_top < lc + 1) {
      for (int b = lane64; b < G; b += 64) up[b] = get(a.tree[par] + tree_off(m, lc + 1) + b);
      wsync();
      up_top = lc + 1;
    }
    for (; up_top < level; ++up_top) {
      const int u = up_top + 1 - (lc + 1);
      const int cnt = G >> u;
      const int o_prev = 2 * G - ((2 * G) >> (u - 1)), o = 2 * G - ((2 * G) >> u);
      for (int i = lane64; i < cnt; i += 64) up[o + i] = pair_mean(up[o_prev + 2 * i], up[o_prev + 2 * i + 1]);
      wsync();
    }
  };
  auto lt_value = [&](int64_t t, int level, int idx) -> double {
    const int par = static_cast<int>(t & 1);
    if (level <= lc + 1) {
      const int lo = kbase >> (level - 1);
      if (idx >= lo && idx < lo + (c >> (level - 1)))
        return lvp(static_cast<int>(t % 3))[2 * c - ((2 * c) >> (level - 1)) + (idx - lo)];
      if (level == lc + 1) return up[idx];
      return get(a.tree[par] + tree_off(m, level) + idx);
    }
    const int u = level - (lc + 1);
    return up[2 * G - ((2 * G) >> u) + idx];
  };
  // this block's part of the island tree of step t (levels 2 .. lc+1 from
  // the island log-weights), published with the ENF records of levels
  // rec_from .. lc+1
  auto publish = [&](int64_t t, int rec_from) {
    const int par = static_cast<int>(t & 1);
    double* lv = lvp(static_cast<int>(t % 3));
    if (c <= 64) {
      double v = (lane64 < c) ? lv[lane64] : ninf();
      for (int l = 2; l <= lc + 1; ++l) {
        const int cnt = c >> (l - 1);
        const int o = 2 * c - ((2 * c) >> (l - 1));
        const double v0 = __shfl(v, (2 * lane64) & 63, 64), v1 = __shfl(v, (2 * lane64 + 1) & 63, 64);
        const double nv = lane64 < cnt ? pair_mean(v0, v1) : ninf();
        if (lane64 < cnt) lv[o + lane64] = nv;
        v = nv;
      }
    } else {
      for (int l = 2; l <= lc + 1; ++l) {
        const int cnt = c >> (l - 1);
        const int o_prev = 2 * c - ((2 * c) >> (l - 2)), o = 2 * c - ((2 * c) >> (l - 1));
        for (int i = lane64; i < cnt; i += 64) lv[o + i] = pair_mean(lv[o_prev + 2 * i], lv[o_prev + 2 * i + 1]);
        wsync();
      }
    }
    wsync();
    for (int l = 1; l <= lc + 1; ++l) {
      const int cnt = c >> (l - 1);
      const int o = 2 * c - ((2 * c) >> (l - 1));
      double* dst = a.tree[par] + tree_off(m, l) + (kbase >> (l - 1));
      for (int i = lane64; i < cnt; i += 64) put(dst + i, lv[o + i]);
    }
    for (int l = rec_from; l <= lc + 1; ++l) {
      const int cnt = c >> (l - 1);
      const int o = 2 * c - ((2 * c) >> (l - 1));
      const EnfRec r = wave_reduce_enf(cnt, [&](int i) { return enf_leaf(lv[o + i]); });
      if (lane64 == 0) {
        double* pl = a.part[par] + static_cast<int64_t>(l - 1) * 3 * G;
        put(pl + bid, r.E);
        put(pl + G + bid, r.a);
        put(pl + 2 * G + bid, r.b);
      }
    }
  };
  // the flag-array grid barrier of forward_body, taken by this wave alone
  auto barrier = [&]() -> bool {
    __builtin_amdgcn_s_waitcnt(0);
    ++epoch;
    if (lane64 == 0) put(&a.bar[bid], epoch);
    // a lane watches the flags of blocks lane, lane + 64, ... (G <= 256):
    // all of them are loaded before any is tested, one round trip per poll
    int ok = 1;
    unsigned spins = 0;
    while (true) {
      unsigned f[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) f[j] = lane64 + 64 * j < G ? get(&a.bar[lane64 + 64 * j]) : epoch;
      if (f[0] >= epoch && f[1] >= epoch && f[2] >= epoch && f[3] >= epoch) break;
      __builtin_amdgcn_s_sleep(1);
      if ((++spins & 1023u) == 0 && (spins > (1u << 24) || get(a.status) != 0)) {
        put(a.status, 1);
        ok = 0;
        break;
      }
    }
    return __all(ok) != 0;
  };
  // Stage 1's records.  This block's level-1 ENF record of step t goes to
  // slot t mod kRingSlots of a ring whose words are NaN until written (into
  // each of the ring's copies, by one lane per copy; the block polls one
  // copy, and what is said here holds copy by copy, a copy's clearings and
  // records being stored by the same lane).  A record is the block's
  // arrival: no flag, and no wait for the record's own stores.  The record
  // of step t goes out one step before its poll (while the decision of step
  // t-1 is taken), so the exchange's latency overlaps a whole step.
  //   Reuse of a slot: beside the record of step t the block clears its
  // entry of slot t+1 mod kRingSlots, last used by step t+1-kRingSlots =
  // t-4.  Every block has read the records of t-4: this block has taken all
  // records of t-2 (the decision before this publication), and each block
  // stored its record of t-2 after its poll of t-4.  The clearing completes
  // before this block's next record is stored (the s_waitcnt below), and a
  // block polls step t+1 only after it has taken this block's record of t,
  // so it sees the cleared slot.
  //   When a decision finds that step t-1 interacts, the record of step t
  // has gone out on the assumption that it does not: every block clears its
  // entry (no block polls step t before deciding t-1) before the barrier of
  // the interaction, and publishes the record again after step t is run
  // again.
  auto ring_entry = [&](int copy, int64_t t) {
    return a.ring + static_cast<int64_t>(copy) * (3 * kRingSlots) * G + (t % kRingSlots) * 3 * G + bid;
  };
  auto publish_rec = [&](int64_t t) {
    if (S == 0) return;
    const EnfRec* lf = s_leaf[t % 3];
    const EnfRec own = wave_reduce_enf(c, [&](int i) { return lf[i]; });
    const EnfRec mine{readlane_f64(own.E, 0), readlane_f64(own.a, 0), readlane_f64(own.b, 0)};
    __builtin_amdgcn_s_waitcnt(0);
    if (lane64 < kRingCopies) {                                 // lane r writes copy r
      double* w = ring_entry(lane64, t);
      put(w, mine.E);
      put(w + G, mine.a);
      put(w + 2 * G, mine.b);
      double* rp = ring_entry(lane64, t + 1);
      const double nan = __longlong_as_double(static_cast<long long>(~0ull));
      put(rp, nan);
      put(rp + G, nan);
      put(rp + 2 * G, nan);
    }
  };
  // this block's record of step t taken back (the step is run again)
  auto retract_rec = [&](int64_t t) {
    if (lane64 < kRingCopies) {
      double* w = ring_entry(lane64, t);
      const double nan = __longlong_as_double(static_cast<long long>(~0ull));
      put(w, nan);
      put(w + G, nan);
      put(w + 2 * G, nan);
    }
  };
  // each lane waits until the records of step t of its blocks (those
  // wave_join_flat assigns it) are complete; they are joined as
  // wave_join_flat joins them
  auto poll_rec = [&](int64_t t, EnfRec& out) -> bool {
    const double* rs = ring_entry(bid & (kRingCopies - 1), t) - bid;
    const int per = G > 64 ? (G >> 6) : 1;                     // blocks per lane: 4, 2 or 1
    const int i0 = G > 64 ? lane64 * per : lane64;
    const int cnt = G > 64 ? per : (lane64 < G ? 1 : 0);
    EnfRec rec[4] = {{ninf(), 0.0, 0.0}, {ninf(), 0.0, 0.0}, {ninf(), 0.0, 0.0}, {ninf(), 0.0, 0.0}};
    const unsigned all = (1u << cnt) - 1u;
    unsigned got = 0;
    unsigned spins = 0;
    int ok = 1;
    while (got != all) {
      // every word of the lane's blocks is loaded before any is tested: the
      // records were sent out a step earlier and are mostly here, so a poll
      // is one round trip, not one per block (a record already taken is
      // read again, unused)
      double e[4], va[4], vb[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const bool want = j < cnt;
        e[j] = want ? get(rs + i0 + j) : 0.0;
        va[j] = want ? get(rs + G + i0 + j) : 0.0;
        vb[j] = want ? get(rs + 2 * G + i0 + j) : 0.0;
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        if (j < cnt && !(got & (1u << j)) && e[j] == e[j] && va[j] == va[j] && vb[j] == vb[j]) {
          rec[j] = EnfRec{e[j], va[j], vb[j]};
          got |= 1u << j;
        }
      }
      if (got == all) break;
      __builtin_amdgcn_s_sleep(1);
      if ((++spins & 1023u) == 0 && (spins > (1u << 24) || get(a.status) != 0)) {
        put(a.status, 1);
        ok = 0;
        break;
      }
    }
    out = wave_join_flat(rec, per, G);
    return __all(ok) != 0;
  };
  // the observations of chunk j (steps j * kYChunk onwards) into s_y[j & 1];
  // observations the host could not check are checked here
  auto load_y = [&](int64_t j) {
    const int dy = a.dy;
    const int64_t n0 = j * kYChunk;
    double* dst = s_y[j & 1];
    bool fin = true;
    for (int i = lane64; i < kYChunk * dy; i += 64) {
      const double v = n0 + i / dy < T ? a.y[n0 * dy + i] : 0.0;
      fin = fin && isfinite(v);
      dst[i] = v;
    }
    if (a.check_y && !fin) put(a.bad_y, 1);
  };
  // resampled blocks of step t from LDS to HBM
  auto write_out = [&](int64_t t) {
    const int par = static_cast<int>(t & 1), sl = static_cast<int>(t % 3);
    Store* xo_blk = static_cast<Store*>(a.x1[par]) + static_cast<int64_t>(kbase) * N * DX;
    for (int64_t w = lane64; w < res_words; w += 64) put(xo_blk + w, res[sl * res_words + w]);
  };
  // Take the records of step t, decide s*_t and walk; sets s_ctl[1] when the
  // run ends here (every island dead, or a wait that did not complete).
  // Stage 1 needs only the blocks' level-1 records; the tree and the other
  // levels' records follow (with a barrier) only when stage 1 interacts,
  // which every block decides alike.  `next_out`: the record of step t+1 has
  // gone out (it is taken back when step t interacts).
  auto control_step = [&](int64_t t, bool next_out) {
    if (S == 0) {                                     // one island: no stages
      if (lane64 == 0) {
        s_ctl[0] = 0;
        if (Rec && tr_sstar) tr_sstar[t] = 0;
        if (Rec && tr_pi) tr_pi[t * m + kbase] = kbase;
      }
      return;
    }
    const int par = static_cast<int>(t & 1);
    EnfRec r1;
    if (!poll_rec(t, r1)) { s_ctl[1] = 1; return; }
    up_top = 0;
    int sstar = 0;
    if constexpr (Rary) {
      // stage u reads tree level (u-1) rb + 1; stage 1 is level 1 as for pairs
      const int rb = a.arity_log2, Sr = S / rb, ar = 1 << rb;
      for (int u = 1; u <= Sr; ++u) {
        const int lv = (u - 1) * rb + 1;
        EnfRec r;
        if (u == 1) {
          r = r1;
        } else if (lv <= lc + 1) {
          const double* ps = a.part[par] + static_cast<int64_t>(lv - 1) * 3 * G;
          r = wave_reduce_enf(G, [&](int i) { return EnfRec{get(ps + i), get(ps + G + i), get(ps + 2 * G + i)}; });
        } else {
          build_upper_to(t, lv);
          const double* lvl = up + 2 * G - ((2 * G) >> (lv - lc - 1));
          r = wave_reduce_enf(G >> (lv - lc - 1), [&](int i) { return enf_leaf(lvl[i]); });
        }
        r = EnfRec{readlane_f64(r.E, 0), readlane_f64(r.a, 0), readlane_f64(r.b, 0)};
        if (u == 1 && r.E == ninf()) {                                // every island dead
          if (bid == 0 && lane64 == 0) *a.out_logz = ninf();
          s_ctl[1] = 1;
          return;
        }
        const double blk = static_cast<double>(1 << (lv - 1));
        const double am = (blk * r.a) * __builtin_ldexp(1.0, -S), bm = (blk * r.b) * __builtin_ldexp(1.0, -S);
        if (!enf_below(am, bm, a.tau)) break;
        sstar = u;
        if (u == 1) {
          if (next_out) retract_rec(t + 1);
          write_out(t);
          publish(t, 2);
          if (!barrier()) { s_ctl[1] = 1; return; }
        }
      }
      if (sstar > 0) {
        if (sstar * rb + 1 > lc + 1) build_upper_to(t, sstar * rb + 1);
        for (int li = lane64; li < c; li += 64) {
          const int k = kbase + li;
          int cur = k;
          // at stage u island cur takes member d of its group with
          // probability W_d / sum W: the first d whose running sum of
          // exp(L_d - max L) exceeds u times the total (the last live member
          // if rounding leaves none; all dead: itself)
          for (int u = sstar; u >= 1; --u) {
            const int p = (u - 1) * rb;
            const int own = (cur >> p) & (ar - 1);
            const int b0 = (cur >> p) - own;
            uint32_t w[4];
            draw4(key, static_cast<uint32_t>(u), static_cast<uint32_t>(cur), static_cast<uint32_t>(t), kTagIsl, 0, w);
            const double uu = uniform53(w[0], w[1]);
            double hi = ninf();
            for (int d = 0; d < ar; ++d) {
              const double v = lt_value(t, p + 1, b0 + d);
              hi = v > hi ? v : hi;
            }
            int pick = own;
            if (hi != ninf()) {
              double tot = 0.0;
              for (int d = 0; d < ar; ++d) tot += dexp(lt_value(t, p + 1, b0 + d) - hi);
              const double thr = uu * tot;
              double run = 0.0;
              int last = own;
              bool found = false;
              for (int d = 0; d < ar && !found; ++d) {
                const double wd = dexp(lt_value(t, p + 1, b0 + d) - hi);
                run += wd;
                if (wd > 0.0) last = d;
                if (thr < run) { pick = d; found = true; }
              }
              if (!found) pick = last;
            }
            cur = (b0 + pick) << p | (cur & ((1 << p) - 1));
          }
          s_src[li] = cur;
          s_lpre[li] = lt_value(t, sstar * rb + 1, k >> (sstar * rb));
        }
      }
      if (lane64 == 0) s_ctl[0] = sstar;
      return;
    }
    for (int s = 1; s <= S; ++s) {
      EnfRec r;
      if (s == 1) {
        r = r1;
      } else if (s <= lc + 1) {
        const double* ps = a.part[par] + static_cast<int64_t>(s - 1) * 3 * G;
        r = wave_reduce_enf(G, [&](int i) { return EnfRec{get(ps + i), get(ps + G + i), get(ps + 2 * G + i)}; });
      } else {
        build_upper_to(t, s);
        const double* lvl = up + 2 * G - ((2 * G) >> (s - lc - 1));
        r = wave_reduce_enf(G >> (s - lc - 1), [&](int i) { return enf_leaf(lvl[i]); });
      }
      // the reduction's result is in lanes below its size: take lane 0's
      r = EnfRec{readlane_f64(r.E, 0), readlane_f64(r.a, 0), readlane_f64(r.b, 0)};
      if (s == 1 && r.E == ninf()) {                                  // every island dead
        if (bid == 0 && lane64 == 0) *a.out_logz = ninf();
        s_ctl[1] = 1;
        return;
      }
      const double blk = static_cast<double>(1 << (s - 1));
      const double am = (blk * r.a) * __builtin_ldexp(1.0, -S), bm = (blk * r.b) * __builtin_ldexp(1.0, -S);   // m = 2^S: scaling by the exact reciprocal is the division
      if (!enf_below(am, bm, a.tau)) break;
      sstar = s;
      if (s == 1) {
        if (next_out) retract_rec(t + 1);
        write_out(t);
        publish(t, 2);
        if (!barrier()) { s_ctl[1] = 1; return; }
      }
    }
    if (sstar > 0) {
      if (sstar + 1 > lc + 1) build_upper_to(t, sstar + 1);
      for (int li = lane64; li < c; li += 64) {
        const int k = kbase + li;
        int cur = k;
        for (int s = sstar; s >= 1; --s) {
          const int pr = cur ^ (1 << (s - 1));
          const double lc_ = lt_value(t, s, cur >> (s - 1));
          const double lp_ = lt_value(t, s, pr >> (s - 1));
          uint32_t w[4];
          draw4(key, static_cast<uint32_t>(s), static_cast<uint32_t>(cur), static_cast<uint32_t>(t), kTagIsl, 0, w);
          if (uniform53(w[0], w[1]) < take_partner_prob(lc_, lp_)) cur = pr;
        }
        s_src[li] = cur;
        s_lpre[li] = lt_value(t, sstar + 1, k >> sstar);
        if (Rec && tr_pi) tr_pi[t * m + k] = cur;
      }
    } else if (Rec && tr_pi) {
      for (int li = lane64; li < c; li += 64) tr_pi[t * m + kbase + li] = kbase + li;
    }
    if (lane64 == 0) {
      s_ctl[0] = sstar;
      if (Rec && tr_sstar) tr_sstar[t] = sstar;
    }
  };

  // τ so small that no stage can ever interact: nothing is exchanged until
  // the final log Zhat (the decisions are s* = 0 by definition)
  const bool never = a.no_interaction;
  auto settle = [&](int64_t t) {
    if (lane64 == 0) {
      s_ctl[0] = 0;
      if (Rec && tr_sstar) tr_sstar[t] = 0;
    }
    if (Rec && tr_pi)
      for (int li = lane64; li < c; li += 64) tr_pi[t * m + kbase + li] = kbase + li;
  };

  // ================= the step loop =================
  // Iteration n runs step n in the workers on the assumption that steps n-1
  // and n-2 do not interact, while the control wave sends out the record of
  // step n-1 and decides step n-2 from the records sent out one iteration
  // earlier.  When step n-2 interacts, steps n-1 and n are run again (n-1
  // from the walk's sources), the record of n-1 going out again beside the
  // second run of n.
  if (ctl) {
    if (lane64 == 0) { s_ctl[0] = 0; s_ctl[1] = 0; }
    load_y(0);
  }
  __syncthreads();
  if (!ctl) run_passes(0, false);
  else if (T > kYChunk) load_y(1);
  __syncthreads();
  if (T > 1) {
    if (ctl) {
      if (!never) publish_rec(0);
    } else {
      run_passes(1, true);
    }
    __syncthreads();
  }
  for (int64_t n = 2; n < T; ++n) {
    if (ctl) {
      if (never) {
        settle(n - 2);
      } else {
        publish_rec(n - 1);
        control_step(n - 2, true);
      }
      // chunk n/64 + 1 into the buffer of chunk n/64 - 1, whose last step
      // (64 (n/64) - 1 = n - 2) this iteration no longer runs
      if (n % kYChunk == 1 && n > kYChunk && n + kYChunk - 1 < T) load_y(n / kYChunk + 1);
    } else {
      run_passes(n, true);
    }
    __syncthreads();
    if (s_ctl[1]) return;
    if (s_ctl[0] > 0) {
      // steps n-1 (from the walk's sources) and n again
      if (!ctl) run_passes(n - 1, false);
      __syncthreads();
      if (ctl) publish_rec(n - 1);
      else run_passes(n, true);
      __syncthreads();
    }
  }
  if (T > 1) {
    // the last decision, s*_{T-2}; no record of step T-1 goes out
    if (ctl) {
      if (never) settle(T - 2);
      else control_step(T - 2, false);
    }
    __syncthreads();
    if (s_ctl[1]) return;
    if (s_ctl[0] > 0) {
      if (!ctl) run_passes(T - 1, false);
      __syncthreads();
    }
  }

  // ---- log Zhat: the root of the island tree after the last weighting ----
  if (!ctl) return;
  publish(T - 1, lc + 2);
  if (!barrier()) return;
  if (bid == 0) {
    up_top = 0;
    build_upper_to(T - 1, S + 1);
    if (lane64 == 0) {
      *a.out_logz = up[2 * G - 2];
      if (Rec && tr_sstar) tr_sstar[T - 1] = 0;
    }
  }
}

template <class Model, typename Store, int PPT, bool Rec, int TPC = 0, bool Rary = false, bool Mult = false>
__global__ __launch_bounds__(kPipeBlock) void forward_pipe_kernel(FwdArgs a) {
  forward_pipe_body<Model, Store, PPT, Rec, TPC, Rary, Mult>(a, static_cast<int>(blockIdx.x));
}

template <class Model, typename Store, int PPT, bool Plain>
__global__ __launch_bounds__(kBlock) void forward_kernel(FwdArgs a) {
  forward_body<Model, Store, PPT, Plain>(a, static_cast<int>(blockIdx.x));
}

// adaptive internal resampling (single problem, traced or not; double states)
template <class Model, typename Store, int PPT>
__global__ __launch_bounds__(kBlock) void forward_adapt_kernel(FwdArgs a) {
  forward_body<Model, Store, PPT, false, false, true>(a, static_cast<int>(blockIdx.x));
}

// multinomial internal resampling (single problem, traced or not)
template <class Model, typename Store, int PPT>
__global__ __launch_bounds__(kBlock) void forward_mult_kernel(FwdArgs a) {
  forward_body<Model, Store, PPT, false, true>(a, static_cast<int>(blockIdx.x));
}

// Several problems in one cooperative launch: block b runs block bmap[b].y of
// problem bmap[b].x; each problem synchronises only its own blocks.
template <class Model, typename Store, int PPT, bool Plain>
__global__ __launch_bounds__(kBlock) void forward_batch_kernel(const FwdArgs* probs, const int2* bmap) {
  const int2 pb = bmap[blockIdx.x];
  forward_body<Model, Store, PPT, Plain>(probs[pb.x], pb.y);
}

// the same with multinomial internal resampling
template <class Model, typename Store, int PPT>
__global__ __launch_bounds__(kBlock) void forward_batch_mult_kernel(const FwdArgs* probs, const int2* bmap) {
  const int2 pb = bmap[blockIdx.x];
  forward_body<Model, Store, PPT, false, true>(probs[pb.x], pb.y);
}

}  // namespace airpf

// ============================================================ host launcher

namespace airpf {

inline int pow2_ceil(int v) { int p = 1; while (p < v) p <<= 1; return p; }
inline int ilog2i(int v) { int s = 0; while ((1 << s) < v) ++s; return s; }

// nothing traced, recorded, replayed or checkpointed: the Plain kernel runs it
inline bool fwd_is_plain(const FwdArgs& a) {
  return !a.tr_sstar && !a.tr_enf && !a.tr_lpost && !a.tr_anc && !a.tr_pi && !a.tr_digest && !a.tr_fmean && !a.tr_lpre && !a.rec_x &&
         !a.rec_anc && !a.ck_x && !a.ck_L && !a.ck_in && a.ck_every == 0 && !a.replay_pi && a.n0 == 0 && a.n1 == a.T;
}

// the pipelined kernel's conditions (besides resampled states resident in
// LDS at its tiling): untraced, teams inside one wave, and a tau at which
// stages can but need not interact (speculation pays); AIRPF_PIPELINE=0
// switches it off
// the score's forward: island maps, s*, entering weights and checkpoints
// kept, nothing else traced or replayed
inline bool fwd_is_score_forward(const FwdArgs& a) {
  return !a.tr_enf && !a.tr_lpost && !a.tr_anc && !a.tr_digest && !a.tr_fmean && !a.rec_x && !a.rec_anc && !a.ck_in &&
         !a.replay_pi && a.n0 == 0 && a.n1 == a.T;
}

inline bool fwd_pipe_candidate(const FwdArgs& a, int TP) {
  if (!(fwd_is_plain(a) || fwd_is_score_forward(a)) || TP > 64 || a.shortcut_all || a.ess_frac > 0.0 ||
      (a.multinomial && (!fwd_is_plain(a) || a.arity_log2 > 1)) ||
      (a.arity_log2 > 1 && !a.no_interaction && !fwd_is_plain(a)))
    return false;
  const char* e = std::getenv("AIRPF_PIPELINE");
  return !(e && e[0] == '0');
}

inline size_t fwd_res_bytes(size_t store_bytes, int dx, int c, int N) {
  const size_t b = 2 * store_bytes * size_t(dx) * size_t(c) * size_t(N);
  return b <= kResidentBudget ? b : 0;
}

// the pipelined kernel keeps three steps' resampled states (the steps being
// decided, sent out and run) and island log-weights
inline size_t pipe_res_bytes(size_t store_bytes, int dx, int c, int N) {
  const size_t b = 3 * store_bytes * size_t(dx) * size_t(c) * size_t(N);
  return b <= 3 * (kResidentBudget / 2) ? b : 0;
}

inline size_t fwd_smem_bytes(size_t store_bytes, int ppt, int dx, int c, int G) {
  const size_t sx = (store_bytes * kBlock * ppt * dx + 15) & ~size_t(15);
  return sx + 4 * size_t(kBlock) * ppt + 8 * 4 * size_t(c) + 8 * 2 * size_t(G);
}

// The largest power-of-two block count G <= min(m / tpb, cap) whose blocks
// (threads each, LDS by smem_of(G)) are all co-resident; 0 if none.
template <class SmemOf>
static int fit_blocks(const void* kern, int threads, const FwdLaunch& L, int m, int tpb, int cap, SmemOf smem_of,
                      size_t* smem_out) {
  int G = m / tpb;
  if (G < 1) G = 1;
  if (G > cap) G = cap;
  G = 1 << ilog2i(G + 1) >> 1;                  // power of two <= G
  for (; G >= 1; G >>= 1) {
    const size_t smem = smem_of(G);
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, threads, smem) != hipSuccess) return 0;
    if (static_cast<long>(per_cu) * L.num_cus >= G) { *smem_out = smem; return G; }
  }
  return 0;
}

template <class Model, typename Store, int PPT>
static hipError_t launch_t(const FwdLaunch& L, FwdArgs a, FwdPlan* plan) {
  const int TP = pow2_ceil((a.N + PPT - 1) / PPT);
  const int tpb = kBlock / TP;
  auto smem_of = [&](int G) {
    const int c = a.m / G;
    return fwd_smem_bytes(sizeof(Store), PPT, Model::DX, c, G) + fwd_res_bytes(sizeof(Store), Model::DX, c, a.N) +
           (a.multinomial ? 16 + 8 * size_t(kBlock) * PPT : 0);     // the cumulative weights of multinomial draws
  };
  auto set_plan = [&](int G, size_t smem) {
    a.TP = TP;
    a.G = G;
    a.c = a.m / G;
    a.lc = ilog2i(a.c);
    a.res_lds = fwd_res_bytes(sizeof(Store), Model::DX, a.c, a.N) > 0;
    plan->ppt = PPT; plan->tp = TP; plan->G = G; plan->c = a.c; plan->smem = smem;
  };
  void* args[] = {&a};
  size_t smem = 0;
  // the pipelined kernel: one five-wave block per CU at most, G <= 256 (its
  // level-1 record wait reads at most four blocks per lane), and the
  // resampled states resident in LDS
  if (fwd_pipe_candidate(a, TP)) {
    const bool plain = fwd_is_plain(a);
    const void* pk = plain ? reinterpret_cast<const void*>(forward_pipe_kernel<Model, Store, PPT, false>)
                           : reinterpret_cast<const void*>(forward_pipe_kernel<Model, Store, PPT, true>);
    // binary32 1-D islands that fill 64- or 32-lane teams: the kernel
    // compiled for that width (same results)
    const bool rary = a.arity_log2 > 1 && !a.no_interaction;
    if (a.multinomial) pk = reinterpret_cast<const void*>(forward_pipe_kernel<Model, Store, PPT, false, 0, false, true>);
    else if (rary) pk = reinterpret_cast<const void*>(forward_pipe_kernel<Model, Store, PPT, false, 0, true>);
    else if constexpr (std::is_same<Store, float>::value && PPT == 4 && Model::DX == 1) {
      if (a.N == 64 * PPT)
        pk = plain ? reinterpret_cast<const void*>(forward_pipe_kernel<Model, Store, PPT, false, 64>)
                   : reinterpret_cast<const void*>(forward_pipe_kernel<Model, Store, PPT, true, 64>);
      else if (a.N == 32 * PPT)
        pk = plain ? reinterpret_cast<const void*>(forward_pipe_kernel<Model, Store, PPT, false, 32>)
                   : reinterpret_cast<const void*>(forward_pipe_kernel<Model, Store, PPT, true, 32>);
    }
    auto pipe_smem_of = [&](int G) {
      const int c = a.m / G;
      return fwd_smem_bytes(sizeof(Store), PPT, Model::DX, c, G) + 8 * 2 * size_t(c) +
             pipe_res_bytes(sizeof(Store), Model::DX, c, a.N) +
             (a.multinomial ? 16 + 8 * size_t(kBlock) * PPT : 0);     // the cumulative weights of multinomial draws
    };
    const int G = fit_blocks(pk, kPipeBlock, L, a.m, tpb, L.max_blocks < 256 ? L.max_blocks : 256, pipe_smem_of, &smem);
    if (G >= 1 && a.m / G <= kMaxIslandsPerBlock && pipe_res_bytes(sizeof(Store), Model::DX, a.m / G, a.N) > 0) {
      set_plan(G, smem);
      if (L.plan_only) return hipSuccess;
      return hipLaunchCooperativeKernel(pk, dim3(G), dim3(kPipeBlock), args, static_cast<unsigned>(smem), L.stream);
    }
  }
  const void* kern = a.multinomial    ? reinterpret_cast<const void*>(forward_mult_kernel<Model, Store, PPT>)
                     : fwd_is_plain(a) ? reinterpret_cast<const void*>(forward_kernel<Model, Store, PPT, true>)
                                       : reinterpret_cast<const void*>(forward_kernel<Model, Store, PPT, false>);
  if (a.ess_frac > 0.0) {
    if constexpr (std::is_same<Store, double>::value) kern = reinterpret_cast<const void*>(forward_adapt_kernel<Model, Store, PPT>);
    else return hipErrorInvalidValue;                           // adaptive runs keep double states
  }
  const int G = fit_blocks(kern, kBlock, L, a.m, tpb, L.max_blocks, smem_of, &smem);
  if (G < 1) return hipErrorCooperativeLaunchTooLarge;
  if (a.m / G > kMaxIslandsPerBlock) return hipErrorInvalidValue;     // islands per block are bounded by the LDS plan
  set_plan(G, smem);
  if (a.ess_frac > 0.0) a.res_lds = 0;        // the adaptive kernel reads every source block from HBM
  if (L.plan_only) return hipSuccess;
  return hipLaunchCooperativeKernel(kern, dim3(G), dim3(kBlock), args, static_cast<unsigned>(smem), L.stream);
}

// particles per lane: the smallest PPT with PPT*DX a multiple of four (a lane
// consumes whole Philox blocks) and at most 256 lanes per island
template <class Model, typename Store>
static hipError_t dispatch_ppt(const FwdLaunch& L, const FwdArgs& a, FwdPlan* plan) {
  constexpr int DX = Model::DX;
  if constexpr (DX % 4 == 0) {
    if (a.N <= 256) return launch_t<Model, Store, 1>(L, a, plan);
    if (a.N <= 512) return launch_t<Model, Store, 2>(L, a, plan);
  } else if constexpr (DX % 2 == 0) {
    if (a.N <= 512) return launch_t<Model, Store, 2>(L, a, plan);
  }
  if (a.N <= 1024) return launch_t<Model, Store, 4>(L, a, plan);
  return launch_t<Model, Store, 8>(L, a, plan);
}

template <class Model, typename Store, int PPT>
static hipError_t batch_fwd_t(const BatchLaunch& L, int* cap) {
  auto kern = L.multinomial ? forward_batch_mult_kernel<Model, Store, PPT>
              : (L.plain ? forward_batch_kernel<Model, Store, PPT, true> : forward_batch_kernel<Model, Store, PPT, false>);
  if (cap) {
    int per_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, kBlock, L.smem);
    *cap = per_cu * L.num_cus;
    return e;
  }
  const void* probs = L.probs;
  const int2* bmap = L.bmap;
  void* args[] = {&probs, &bmap};
  return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(kern), dim3(L.blocks), dim3(kBlock), args,
                                    static_cast<unsigned>(L.smem), L.stream);
}

template <class Model, typename Store>
static hipError_t batch_fwd_ppt(const BatchLaunch& L, int* cap) {
  switch (L.ppt) {              // the items' teams were sized for it
    case 1: if constexpr (Model::DX % 4 == 0) return batch_fwd_t<Model, Store, 1>(L, cap); break;
    case 2: if constexpr (Model::DX % 2 == 0) return batch_fwd_t<Model, Store, 2>(L, cap); break;
    case 4: return batch_fwd_t<Model, Store, 4>(L, cap);
    case 8: return batch_fwd_t<Model, Store, 8>(L, cap);
  }
  return hipErrorInvalidValue;
}

// one model's launches in both storage precisions (each model's kernels are
// compiled in a translation unit of their own)
template <class Model>
hipError_t fwd_launch_model(const FwdLaunch& L, const FwdArgs& a, FwdPlan* plan) {
  if constexpr (Model::kWordNoise) return dispatch_ppt<Model, double>(L, a, plan);   // word-driven models: double states
  else return L.fp64 ? dispatch_ppt<Model, double>(L, a, plan) : dispatch_ppt<Model, float>(L, a, plan);
}
template <class Model>
hipError_t fwd_batch_model(const BatchLaunch& L, int* cap) {
  return L.fp64 ? batch_fwd_ppt<Model, double>(L, cap) : batch_fwd_ppt<Model, float>(L, cap);
}

hipError_t fwd_launch_lg1(const FwdLaunch& L, const FwdArgs& a, FwdPlan* plan);
hipError_t fwd_batch_lg1(const BatchLaunch& L, int* cap);
hipError_t fwd_launch_sv(const FwdLaunch& L, const FwdArgs& a, FwdPlan* plan);
hipError_t fwd_launch_bin(const FwdLaunch& L, const FwdArgs& a, FwdPlan* plan);
hipError_t fwd_launch_bcp(const FwdLaunch& L, const FwdArgs& a, FwdPlan* plan);
hipError_t fwd_batch_sv(const BatchLaunch& L, int* cap);
hipError_t fwd_launch_lgd2(const FwdLaunch& L, const FwdArgs& a, FwdPlan* plan);
hipError_t fwd_batch_lgd2(const BatchLaunch& L, int* cap);
hipError_t fwd_launch_lgd3(const FwdLaunch& L, const FwdArgs& a, FwdPlan* plan);
hipError_t fwd_batch_lgd3(const BatchLaunch& L, int* cap);
hipError_t fwd_launch_lgd4(const FwdLaunch& L, const FwdArgs& a, FwdPlan* plan);
hipError_t fwd_batch_lgd4(const BatchLaunch& L, int* cap);
hipError_t fwd_launch_lgd8(const FwdLaunch& L, const FwdArgs& a, FwdPlan* plan);
hipError_t fwd_batch_lgd8(const BatchLaunch& L, int* cap);

}  // namespace airpf
