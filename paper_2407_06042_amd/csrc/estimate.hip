// Estimators on the final samples (Algorithm 2, steps after sampling).
//
// One workgroup per instance.  For every chain's final state x^[s] (the sample
// list of Section IV-A) the kernel recomputes the residual r = y - H x from the
// inputs, E = ||r||^2, f = -E/sigma^2 and c = H^H r.  Moving coordinate n of a
// sample from level k_n to level k (e = k - k_n, real step d = 2 s e) changes f by
//     delta(e) = (2 d c_n - d^2 ||h_m||^2) / sigma^2 = e (a_n - a2_m e),
//     a_n = 4 s c_n / sigma^2,  a2_m = 4 s^2 ||h_m||^2 / sigma^2,
// which gives, per bit (eq. llr_is in the log-sum-exp form of eq. llr_simple,
// F(a) = log(1 + e^a) evaluated exactly)
//     L = LSE_s[((tau-1)/tau) F+ - F(-g)] - LSE_s[((tau-1)/tau) F- - F(g)],  g = (F+ - F-)/tau,
// and per antenna and point a = (kI, kQ) the symbol-level IS estimate
//     p(a) propto sum_s pi_a(a | x^[s]_-m) exp(((tau-1)/tau) f(x^[s]_{m<-a}))
//          = sum_s exp(((tau-1)/tau) f_s + delta_I(kI) + delta_Q(kQ) - lse_I - lse_Q),
// lse_{I,Q} = log sum_k exp(delta_{I,Q}(k)/tau): the I/Q parts separate because
// the real-equivalent columns of one antenna are orthogonal.  The hard decision
// is the chain whose tracked best state has the smallest recomputed energy.
//
// Chains are processed in chunks staged in LDS; every output keeps a running
// log-sum-exp in registers across chunks.  A thread owns (antenna, kI) and the
// Q points (kI, 0..Q-1), so the inner loop has Q independent accumulators.
#include "common.hpp"

namespace dmala {

__device__ __forceinline__ float fexp(float x) { return __builtin_amdgcn_exp2f(x * 1.4426950408889634f); }
__device__ __forceinline__ float fex2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float flg2(float x) { return __builtin_amdgcn_logf(x); }
__device__ __forceinline__ double fex2(double x) { return exp2(x); }
__device__ __forceinline__ double flg2(double x) { return log2(x); }
__device__ __forceinline__ float flog(float x) { return __builtin_amdgcn_logf(x) * 0.6931471805599453f; }
__device__ __forceinline__ double fexp(double x) { return exp(x); }
__device__ __forceinline__ double flog(double x) { return log(x); }

template <typename R>
struct OnlineLse {
  R mx, sum;
  __device__ OnlineLse() : mx(-INFINITY), sum(R(0)) {}
  __device__ __forceinline__ void add(R v) {  // branch-free: both lanes of a divergent update cost the same
    const R m2 = fmax(v, mx);
    sum = sum * fexp(mx - m2) + fexp(v - m2);
    mx = m2;
  }
  __device__ R value() const { return mx + flog(sum); }
};

constexpr int kLlrPerThread = 4;  // bits per instance <= 128 antennas x 8 bits = 4 x 256 threads
// Workgroups of 1024 threads serve instances with more than 256 (antenna, kI) rows: fewer row
// blocks, so the chain chunks are staged (residuals, H^H r) fewer times, and 16 waves per CU.

// Exchanges inside groups of Q consecutive lanes (Q <= 16, so a group never straddles a 32-lane
// half) by ds_swizzle in its bit mode: lane j reads lane ((j & and) | or) ^ xor of its half, an
// immediate pattern, so no lane-address registers are needed.
template <int PAT> __device__ __forceinline__ float swz(float x) {
  return __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(x), PAT));
}
template <int PAT> __device__ __forceinline__ double swz(double x) {
  const long long u = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_ds_swizzle((int)u, PAT), hi = __builtin_amdgcn_ds_swizzle((int)(u >> 32), PAT);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
// x of every member of the lane's group, in member order
template <int Q, int K = 0, typename R> __device__ __forceinline__ void group_gather(R x, R (&out)[Q]) {
  out[K] = swz<(0x1F & ~(Q - 1)) | (K << 5)>(x);
  if constexpr (K + 1 < Q) group_gather<Q, K + 1>(x, out);
}
// the largest x of the group (a butterfly)
template <int Q, int O = 1, typename R> __device__ __forceinline__ R group_max(R x) {
  if constexpr (O < Q) return group_max<Q, 2 * O>(fmax(x, swz<0x1F | (O << 10)>(x)));
  else return x;
}

// Per (chain, antenna) values staged in LDS.
template <typename R>
struct CM {
  R aI, aQ, base;  // base = ((tau-1)/tau) f_s - lse_I - lse_Q
  int kI, kQ;
};

template <typename R, int Q, bool SH, int BS>
__device__ __forceinline__ void estimate_body(const EstArgs& a, const int b) {
  constexpr int M = Q * Q;
  constexpr int NB = Q == 2 ? 1 : (Q == 4 ? 2 : (Q == 8 ? 3 : 4));
  const int tid = threadIdx.x, nth = blockDim.x;
  const int nt = a.nt, nr = a.nr, C = a.C, Npad = a.Npad, N = a.N, CH = a.chunk;
  const InstDesc dsc = inst_desc(a.desc, b, nt, nr, M, C);
  const R* Hg = (const R*)a.H + 2 * dsc.h_off;
  const R* y = (const R*)a.y + 2 * dsc.y_off;
  const InstParams ip = *(const InstParams*)(a.ws_inst + (size_t)b * a.inst_stride);
  if (ip.nonfinite) {
    // a flagged instance (see the setup kernel): no samples to estimate from; symbols -1,
    // every other output NaN (the whole workgroup leaves here)
    const float nan = __builtin_nanf("");
    for (int m = tid; m < nt; m += nth)
      if (a.symbols) a.symbols[dsc.sym_off + m] = -1;
    for (int e = tid; e < nt * M; e += nth) {
      if (a.marginals) a.marginals[dsc.marg_off + e] = nan;
      if (a.marginals_mc) a.marginals_mc[dsc.marg_off + e] = nan;
    }
    for (int e = tid; e < nt * 2 * NB; e += nth)
      if (a.llrs) a.llrs[dsc.llr_off + e] = nan;
    if (a.best_energy && tid == 0) a.best_energy[dsc.orig] = nan;
    return;
  }
  const R s = (R)ip.s, tau = (R)ip.tau;
  const R inv_s2 = R(1) / (R)ip.sigma2, inv_tau = R(1) / tau;
  const R cw = (tau - R(1)) * inv_tau;
  const R kA = R(-2) * tau * R(0.69314718055994530942);
  const StateOff so = state_offsets(a.Cpad, Npad);
  const unsigned char* st = a.ws_state + (size_t)b * a.state_stride;
  const int8_t* K = (const int8_t*)(st + so.k);
  const int8_t* Kb = (const int8_t*)(st + so.kbest);

  extern __shared__ __attribute__((aligned(16))) unsigned char esm[];
  CM<R>* cm = (CM<R>*)esm;                           // CH x nt
  const int lrs = 2 * nr + 2;                        // residual row stride (one pad entry: chain-strided reads
                                                     // of one column hit distinct banks)
  R* rs = (R*)(cm + (size_t)CH * nt);                // CH x nr complex residuals of the final states
  R* rb2 = rs + (size_t)CH * lrs;                    // CH x nr |residual|^2 of the best states
  R* fs = rb2 + (size_t)CH * nr;                     // CH
  R* ebs = fs + CH;                                  // CH
  R* a2 = ebs + CH;                                  // nt
  R* ys = a2 + nt;                                   // nr complex: y + s (Q-1) sum_m h_m
  int8_t* Ks = (int8_t*)(ys + 2 * nr);               // CH x N
  int8_t* Kbs = Ks + (size_t)CH * N;                 // CH x N
  __shared__ R best_e;
  __shared__ int best_c;
  __shared__ unsigned char dupf[1024];   // list LLRs: chain repeats an earlier chain's final state
  // H is read many times per element: stage it in LDS when it fits, transposed
  // with a padded row (Ht[i][m], leading dimension nt + 1) so that both the
  // row-wise (residual) and the column-wise (H^H r) sweeps are conflict-free.
  const int ldh = nt + 1;
  // (an offset from the LDS array itself: a round trip through an integer address
  // would leave a generic pointer, and flat loads, for every read of H)
  const size_t ht_off = ((size_t)((const unsigned char*)(Kbs + (size_t)CH * N) - esm) + 15) & ~(size_t)15;
  R* Ht = (R*)(esm + ht_off);
  if constexpr (SH) {
    for (int e = tid; e < nt * nr; e += nth) {
      const int m = e / nr, i = e % nr;
      Ht[2 * (i * ldh + m)] = Hg[2 * (size_t)e];
      Ht[2 * (i * ldh + m) + 1] = Hg[2 * (size_t)e + 1];
    }
    __syncthreads();
  }
  auto hre = [&](int m, int i) -> R { if constexpr (SH) return Ht[2 * (i * ldh + m)]; else return Hg[2 * ((size_t)m * nr + i)]; };
  auto him = [&](int m, int i) -> R { if constexpr (SH) return Ht[2 * (i * ldh + m) + 1]; else return Hg[2 * ((size_t)m * nr + i) + 1]; };

  // With the symbol x_m = s ((2 kI - Q + 1) + j (2 kQ - Q + 1)) of level indices k the
  // residual is r = y - H x = y' - 2 s H k, k_m = kI + j kQ, y' = y + s (Q - 1) (1 + j)
  // sum_m h_m: the level indices enter the products directly.
  for (int i = tid; i < nr; i += nth) {
    R sr = 0, si = 0;
    for (int m = 0; m < nt; ++m) { sr += hre(m, i) - him(m, i); si += hre(m, i) + him(m, i); }
    ys[2 * i] = y[2 * i] + s * R(Q - 1) * sr;
    ys[2 * i + 1] = y[2 * i + 1] + s * R(Q - 1) * si;
  }
  for (int m = tid; m < nt; m += nth) {
    R g = 0;
    for (int i = 0; i < nr; ++i) {
      const R hr = hre(m, i), hi = him(m, i);
      g += hr * hr + hi * hi;
    }
    a2[m] = R(4) * s * s * g * inv_s2;
  }
  if (tid == 0) { best_e = R(INFINITY); best_c = 0; }
  const int mode = a.llr_mode;
  if (mode == 1 && a.llrs) {
    // the list holds distinct samples: flag every chain whose first N levels equal an earlier chain's
    const int nw = (N + 3) >> 2;
    for (int c = tid; c < C; c += nth) {
      const uint32_t* kc = (const uint32_t*)(K + (size_t)c * Npad);
      bool dup = false;
      for (int c2 = 0; c2 < c && !dup; ++c2) {
        const uint32_t* k2 = (const uint32_t*)(K + (size_t)c2 * Npad);
        bool same = true;
        for (int w = 0; w < nw; ++w) {
          const int valid = N - 4 * w;
          const uint32_t msk = valid >= 4 ? 0xFFFFFFFFu : ((1u << (8 * valid)) - 1u);
          same = same && ((kc[w] ^ k2[w]) & msk) == 0u;
        }
        dup = same;
      }
      dupf[c] = dup ? 1 : 0;
    }
  }

  // ownership: marginal rows (m, kI), in blocks of one row per thread, and bits (m, ax, bit)
  const int n_rows = nt * Q, n_llr = nt * 2 * NB;
  const int n_rb = (n_rows + nth - 1) / nth;
  const bool single_chunk = CH >= C;
  const bool want_mc = a.marginals_mc != nullptr;
  OnlineLse<R> lnum[kLlrPerThread], lden[kLlrPerThread];
  int cplus[kLlrPerThread];
#pragma unroll
  for (int q = 0; q < kLlrPerThread; ++q) cplus[q] = 0;

  for (int rb = 0; rb < n_rb; ++rb) {
    const int row = rb * nth + tid;
    // row sums sum_c 2^(v_c(kQ) - Mx) (log2 units) with one running maximum Mx for the
    // row: a point more than 2^-126 below the row's largest term underflows to zero,
    // as it would in the normalised marginal anyway
    R Mx = R(-INFINITY), sums[Q];
#pragma unroll
    for (int j = 0; j < Q; ++j) sums[j] = R(0);
    int cnt[Q];
#pragma unroll
    for (int j = 0; j < Q; ++j) cnt[j] = 0;

    for (int c0 = 0; c0 < C; c0 += CH) {
      const int ch = C - c0 < CH ? C - c0 : CH;
      if (!single_chunk || rb == 0) {
        __syncthreads();
        for (int it = tid; it < ch * N; it += nth) {
          const int c = it / N, n = it % N;
          Ks[it] = K[(size_t)(c0 + c) * Npad + n];
          Kbs[it] = Kb[(size_t)(c0 + c) * Npad + n];
        }
        __syncthreads();
        // residuals of the final and of the best states
        if constexpr (std::is_same<R, float>::value && BS >= 512) {
          // (the 256-thread workgroups, held to 96 registers, keep the loop below)
          // On the float32 matrix cores (v_mfma_f32_16x16x4f32: float32 H times the integer
          // level indices): [Re r; Im r] = y' - 2 s [Hr -Hi; Hi Hr] k over the real dimensions
          // n = 2m (kI of antenna m), 2m + 1 (kQ), so that B[n][c] is the staged level byte of
          // chain c.  A unit is one 16-row tile of receive antennas (its real and imaginary rows)
          // and one 16-chain tile, for the final and the best states together; lane l holds
          // A[l % 16][4 s + l / 16], B[4 s + l / 16][l % 16] and the outputs at rows 4 (l / 16) + j.
          typedef float f32x4 __attribute__((ext_vector_type(4)));
          // With at least twice as many waves as units (1024-thread workgroups), every unit's K
          // steps are split between two waves (otherwise half the waves would idle): the second
          // half's accumulators go through the per-(chain, antenna) array, unused until the
          // normalisers below, and are added to the first half's in a fixed order.  (In the
          // 512-thread workgroups the split form's registers would cost the second workgroup per CU.)
          bool ksplit = false;
          if constexpr (BS >= 1024) {
            const int lane = tid & 63, wv = tid >> 6, nwv = nth >> 6;
            const int nrt = (nr + 15) >> 4, nct = (ch + 15) >> 4, ksteps = (N + 3) >> 2, units = nrt * nct;
            ksplit = 2 * units <= nwv && (size_t)units * 64 * 16 * sizeof(float) <= (size_t)ch * nt * sizeof(CM<R>);
            if (ksplit) {
              constexpr int kU = 2;
              const int uu = wv % units, kh = wv / units;   // one item per wave
              const int half = ((ksteps + 1) / 2 + kU - 1) / kU * kU;
              const int st_a = kh ? half : 0, st_b = kh ? ksteps : half;
              const int rt = uu % nrt, ct = uu / nrt;
              const int ia = 16 * rt + (lane & 15), c = 16 * ct + (lane & 15);
              const int iac = ia < nr ? ia : nr - 1, cc = c < ch ? c : ch - 1;
              f32x4 fre = {0.f, 0.f, 0.f, 0.f}, fim = fre, bre = fre, bim = fre;
              for (int st0 = st_a; kh < 2 && st0 < st_b; st0 += kU) {
                R hr0[kU], hi0[kU];
                uint8_t kf0[kU], kb0[kU];
#pragma unroll
                for (int u = 0; u < kU; ++u) {
                  const int n = 4 * (st0 + u) + (lane >> 4), nc = n < N ? n : N - 1, m = nc >> 1;
                  hr0[u] = hre(m, iac);
                  hi0[u] = him(m, iac);
                  kf0[u] = (uint8_t)Ks[cc * N + nc];
                  kb0[u] = (uint8_t)Kbs[cc * N + nc];
                }
#pragma unroll
                for (int u = 0; u < kU; ++u) {
                  // steps past N or past this half's end: zero
                  const int n = 4 * (st0 + u) + (lane >> 4);
                  const bool kin = n < N && st0 + u < st_b;
                  const bool aok = kin && ia < nr, bok = kin && c < ch;
                  const R hr = aok ? hr0[u] : R(0), hi = aok ? hi0[u] : R(0);
                  const R are = (n & 1) ? -hi : hr, aim = (n & 1) ? hr : hi;
                  const R kf = bok ? R(kf0[u]) : R(0), kb = bok ? R(kb0[u]) : R(0);
                  fre = __builtin_amdgcn_mfma_f32_16x16x4f32(are, kf, fre, 0, 0, 0);
                  fim = __builtin_amdgcn_mfma_f32_16x16x4f32(aim, kf, fim, 0, 0, 0);
                  bre = __builtin_amdgcn_mfma_f32_16x16x4f32(are, kb, bre, 0, 0, 0);
                  bim = __builtin_amdgcn_mfma_f32_16x16x4f32(aim, kb, bim, 0, 0, 0);
                }
              }
              float* part = (float*)cm + (size_t)uu * 64 * 16;
              if (kh == 1) {
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                  part[(0 + j) * 64 + lane] = fre[j];
                  part[(4 + j) * 64 + lane] = fim[j];
                  part[(8 + j) * 64 + lane] = bre[j];
                  part[(12 + j) * 64 + lane] = bim[j];
                }
              }
              __syncthreads();
              if (kh == 0) {
                const R s2 = R(2) * s;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                  const int i = 16 * rt + 4 * (lane >> 4) + j;
                  const float pre = fre[j] + part[(0 + j) * 64 + lane], pim = fim[j] + part[(4 + j) * 64 + lane];
                  const float pbr = bre[j] + part[(8 + j) * 64 + lane], pbi = bim[j] + part[(12 + j) * 64 + lane];
                  if (i < nr && c < ch) {
                    rs[c * lrs + 2 * i] = ys[2 * i] - s2 * pre;
                    rs[c * lrs + 2 * i + 1] = ys[2 * i + 1] - s2 * pim;
                    const R br = ys[2 * i] - s2 * pbr, bi = ys[2 * i + 1] - s2 * pbi;
                    rb2[c * nr + i] = br * br + bi * bi;
                  }
                }
              }
            }
          }
          if (!ksplit) {
            const int lane = tid & 63, nrt = (nr + 15) >> 4, nct = (ch + 15) >> 4, ksteps = (N + 3) >> 2;
            const R s2 = R(2) * s;
            for (int u = tid >> 6; u < nrt * nct; u += nth >> 6) {
              const int rt = u % nrt, ct = u / nrt;
              const int ia = 16 * rt + (lane & 15), c = 16 * ct + (lane & 15);
              // every load in bounds (indices clamped, values masked after), so that none is predicated
              const int iac = ia < nr ? ia : nr - 1, cc = c < ch ? c : ch - 1;
              f32x4 fre = {0.f, 0.f, 0.f, 0.f}, fim = fre, bre = fre, bim = fre;
              // two K steps per pass: all their loads issue before the first product
              constexpr int kU = 2;
              for (int st0 = 0; st0 < ksteps; st0 += kU) {
                R hr0[kU], hi0[kU];
                uint8_t kf0[kU], kb0[kU];
#pragma unroll
                for (int u = 0; u < kU; ++u) {
                  const int n = 4 * (st0 + u) + (lane >> 4), nc = n < N ? n : N - 1, m = nc >> 1;
                  hr0[u] = hre(m, iac);
                  hi0[u] = him(m, iac);
                  kf0[u] = (uint8_t)Ks[cc * N + nc];
                  kb0[u] = (uint8_t)Kbs[cc * N + nc];
                }
#pragma unroll
                for (int u = 0; u < kU; ++u) {
                  const int n = 4 * (st0 + u) + (lane >> 4);   // n >= N (K padding, steps past the end): zero
                  const bool aok = n < N && ia < nr, bok = n < N && c < ch;
                  const R hr = aok ? hr0[u] : R(0), hi = aok ? hi0[u] : R(0);
                  const R are = (n & 1) ? -hi : hr, aim = (n & 1) ? hr : hi;
                  const R kf = bok ? R(kf0[u]) : R(0), kb = bok ? R(kb0[u]) : R(0);
                  fre = __builtin_amdgcn_mfma_f32_16x16x4f32(are, kf, fre, 0, 0, 0);
                  fim = __builtin_amdgcn_mfma_f32_16x16x4f32(aim, kf, fim, 0, 0, 0);
                  bre = __builtin_amdgcn_mfma_f32_16x16x4f32(are, kb, bre, 0, 0, 0);
                  bim = __builtin_amdgcn_mfma_f32_16x16x4f32(aim, kb, bim, 0, 0, 0);
                }
              }
#pragma unroll
              for (int j = 0; j < 4; ++j) {
                const int i = 16 * rt + 4 * (lane >> 4) + j;
                if (i < nr && c < ch) {
                  rs[c * lrs + 2 * i] = ys[2 * i] - s2 * fre[j];
                  rs[c * lrs + 2 * i + 1] = ys[2 * i + 1] - s2 * fim[j];
                  const R br = ys[2 * i] - s2 * bre[j], bi = ys[2 * i + 1] - s2 * bim[j];
                  rb2[c * nr + i] = br * br + bi * bi;
                }
              }
            }
          }
        } else
        for (int it = tid; it < ch * nr; it += nth) {
          const int c = it / nr, i = it % nr;
          const uint16_t* kf = (const uint16_t*)(Ks + c * N);   // (k_I, k_Q) of antenna m, as bytes
          const uint16_t* kb = (const uint16_t*)(Kbs + c * N);
          R re = 0, im = 0, bre = 0, bim = 0;
          for (int m = 0; m < nt; ++m) {
            const R hr = hre(m, i), hi = him(m, i);
            const uint32_t f = kf[m], g = kb[m];
            const R xr = R(f & 0xFFu), xi = R(f >> 8), br = R(g & 0xFFu), bi = R(g >> 8);
            re += hr * xr - hi * xi;
            im += hr * xi + hi * xr;
            bre += hr * br - hi * bi;
            bim += hr * bi + hi * br;
          }
          const R s2 = R(2) * s;
          re = ys[2 * i] - s2 * re;
          im = ys[2 * i + 1] - s2 * im;
          bre = ys[2 * i] - s2 * bre;
          bim = ys[2 * i + 1] - s2 * bim;
          rs[c * lrs + 2 * i] = re;
          rs[c * lrs + 2 * i + 1] = im;
          rb2[it] = bre * bre + bim * bim;
        }
        __syncthreads();
        for (int c = tid; c < ch; c += nth) {
          R e = 0, eb = 0;
          for (int i = 0; i < nr; ++i) {
            e += rs[c * lrs + 2 * i] * rs[c * lrs + 2 * i] + rs[c * lrs + 2 * i + 1] * rs[c * lrs + 2 * i + 1];
            eb += rb2[c * nr + i];
          }
          fs[c] = -e * inv_s2;
          ebs[c] = eb;
        }
        __syncthreads();
        // per (chain, antenna): H^H r, the per-axis log normalisers, the base term.  With H
        // in LDS consecutive lanes take consecutive antennas (conflict-free columns of Ht);
        // with H in global memory they take consecutive chains, so that the lanes of one
        // antenna share each cache line of its column
        for (int it = tid; it < ch * nt; it += nth) {
          const int c = SH ? it / nt : it % ch, m = SH ? it % nt : it / ch;
          CM<R> v;
          if constexpr (std::is_same<R, float>::value) {
            // from the sampler's energy gradient at the final state,
            // g = 2 s log2(e) (G x - z) / (tau sigma^2) = -2 s log2(e) H^H r / (tau sigma^2):
            // 4 s (H^H r) / sigma^2 = -2 tau ln(2) g
            const float* egc = (const float*)(st + so.eg) + (size_t)(c0 + c) * Npad;
            v.aI = kA * egc[2 * m];
            v.aQ = kA * egc[2 * m + 1];
          } else {
            R re = 0, im = 0;
            for (int i = 0; i < nr; ++i) {
              const R hr = hre(m, i), hi = him(m, i);
              const R rr = rs[c * lrs + 2 * i], ri = rs[c * lrs + 2 * i + 1];
              re += hr * rr + hi * ri;
              im += hr * ri - hi * rr;
            }
            v.aI = R(4) * s * re * inv_s2;
            v.aQ = R(4) * s * im * inv_s2;
          }
          v.kI = Ks[c * N + 2 * m];
          v.kQ = Ks[c * N + 2 * m + 1];
          if constexpr (std::is_same<R, float>::value) {
            // per-axis log normalisers over the Q levels, accumulated in log2 units (no scaling
            // before each exponential); the level offsets are exact float differences
            const R sc = inv_tau * R(1.4426950408889634);
            const R q2s = a2[m] * sc, aIs = v.aI * sc, aQs = v.aQ * sc;
            const R kIf = R(v.kI), kQf = R(v.kQ);
            R mi = R(-INFINITY), mq = R(-INFINITY), si = R(0), sq = R(0);
#pragma unroll
            for (int k = 0; k < Q; ++k) {
              const R eI = R(k) - kIf, eQ = R(k) - kQf;
              const R ti = eI * (aIs - q2s * eI), tq = eQ * (aQs - q2s * eQ);
              const R ni = fmax(mi, ti), nq = fmax(mq, tq);
              si = si * fex2(mi - ni) + fex2(ti - ni);
              sq = sq * fex2(mq - nq) + fex2(tq - nq);
              mi = ni;
              mq = nq;
            }
            v.base = cw * fs[c] - (mi + flg2(si) + mq + flg2(sq)) * R(0.6931471805599453);
          } else {
            const R q2 = a2[m];
            OnlineLse<R> li, lq;
#pragma unroll
            for (int k = 0; k < Q; ++k) {
              const R eI = R(k - v.kI), eQ = R(k - v.kQ);
              li.add(eI * (v.aI - q2 * eI) * inv_tau);
              lq.add(eQ * (v.aQ - q2 * eQ) * inv_tau);
            }
            v.base = cw * fs[c] - li.value() - lq.value();
          }
          cm[c * nt + m] = v;
        }
        if (tid == 0 && rb == 0) {
          for (int c = 0; c < ch; ++c)
            if (ebs[c] < best_e) { best_e = ebs[c]; best_c = c0 + c; }
        }
        __syncthreads();
      }

      // symbol marginals and the plain Monte Carlo histogram: row (m, kI).  For chain c the row's
      // terms are b0 + B(kQ), the kI part b0 plus a kQ part B shared by the Q rows of antenna m,
      // which sit in Q consecutive lanes: lane kI of the group forms B(kQ = kI) and its
      // exponential relative to the largest B once, and the group exchanges those Q values by
      // shuffles, so that a row takes three exponentials per chain instead of Q + 1.  The level
      // offsets are differences of small integers, exact in floating point.
      if (row < n_rows) {
        const int m = row / Q, kIt = row % Q;
        const R q2 = a2[m];
        const R l2e = R(1.4426950408889634), q2l = q2 * l2e;
        for (int c = 0; c < ch; ++c) {
          const CM<R> v = cm[c * nt + m];
          const R eI = R(kIt) - R(v.kI), eQ = R(kIt) - R(v.kQ);
          const R b0 = (v.base + eI * (v.aI - q2 * eI)) * l2e;
          const R bq = eQ * (v.aQ * l2e - q2l * eQ);       // B(kQ = kIt)
          const R bmax = group_max<Q>(bq);
          R eqs[Q];
          group_gather<Q>(fex2(bq - bmax), eqs);
          const R lm = b0 + bmax;                          // the row's largest term for chain c
          const R Mn = fmax(lm, Mx);
          const R sc = fex2(Mx - Mn), w = fex2(lm - Mn);
#pragma unroll
          for (int kQt = 0; kQt < Q; ++kQt) sums[kQt] = sums[kQt] * sc + w * eqs[kQt];
          Mx = Mn;
          if (want_mc) {
#pragma unroll
            for (int kQt = 0; kQt < Q; ++kQt) cnt[kQt] += (v.kI == kIt && v.kQ == kQt) ? 1 : 0;
          }
        }
      }
      // bit LLRs: item (m, ax, bit)
      if (rb == 0) {
#pragma unroll
        for (int q = 0; q < kLlrPerThread; ++q) {
          const int it = tid + q * nth;
          if (it < n_llr) {
            const int m = it / (2 * NB), ax = (it / NB) % 2, bit = it % NB;
            const int mask = 1 << (NB - 1 - bit);
            const R q2 = a2[m];
            // one loop per form (the form is uniform: no branch inside the chain loop)
            if (mode == 0) {
              for (int c = 0; c < ch; ++c) {
                const CM<R> v = cm[c * nt + m];
                const int k = ax ? v.kQ : v.kI;
                const R av = ax ? v.aQ : v.aI;
                // the level with this Gray bit cleared (ep) or set (em), as an offset from k: changing
                // Gray bit j of k flips the binary bits j..0, and one of the two is k itself
                const bool gb = ((k ^ (k >> 1)) & mask) != 0;
                const R d = R((k ^ (2 * mask - 1)) - k);
                const R ep = gb ? d : R(0), em = gb ? R(0) : d;
                const R Fp = fs[c] + ep * (av - q2 * ep);
                const R Fm = fs[c] + em * (av - q2 * em);
                const R gm = (Fp - Fm) * inv_tau;
                // F(gm) and F(-gm), F(a) = log(1 + e^a), share log(1 + e^-|gm|) and differ by
                // max(gm, 0) vs max(-gm, 0)
                const R l1 = flog(R(1) + fexp(-fabs(gm)));
                lnum[q].add(cw * Fp - ((gm < R(0) ? -gm : R(0)) + l1));
                lden[q].add(cw * Fm - ((gm > R(0) ? gm : R(0)) + l1));
              }
            } else if (mode == 1) {
              for (int c = 0; c < ch; ++c) {
                const CM<R> v = cm[c * nt + m];
                const int k = ax ? v.kQ : v.kI;
                const bool plus = ((k ^ (k >> 1)) & mask) == 0;   // label bit 0 <-> b = +1
                if (!dupf[c0 + c]) {
                  if (plus) lnum[q].add(fs[c]);
                  else lden[q].add(fs[c]);
                }
              }
            } else {
              for (int c = 0; c < ch; ++c) {
                const CM<R> v = cm[c * nt + m];
                const int k = ax ? v.kQ : v.kI;
                cplus[q] += (((k ^ (k >> 1)) & mask) == 0) ? 1 : 0;
              }
            }
          }
        }
      }
    }
    // normalise over the M points of antenna m: its Q rows sit in Q consecutive
    // lanes of one wavefront, so the log-sum-exp is a Q-lane butterfly
    {
      R lv[Q];
      R mx = R(-INFINITY);
#pragma unroll
      for (int j = 0; j < Q; ++j) {
        lv[j] = (Mx + flg2(sums[j])) * R(0.6931471805599453);
        mx = lv[j] > mx ? lv[j] : mx;
      }
#pragma unroll
      for (int off = 1; off < Q; off <<= 1) { const R o = __shfl_xor(mx, off); mx = o > mx ? o : mx; }
      R sm = R(0);
#pragma unroll
      for (int j = 0; j < Q; ++j) sm += fexp(lv[j] - mx);
#pragma unroll
      for (int off = 1; off < Q; off <<= 1) sm += __shfl_xor(sm, off);
      if (row < n_rows) {
        const int m = row / Q, kIt = row % Q;
        const R inv = R(1) / sm;
        if (a.marginals) {
#pragma unroll
          for (int j = 0; j < Q; ++j) a.marginals[dsc.marg_off + (size_t)m * M + kIt * Q + j] = (float)(fexp(lv[j] - mx) * inv);
        }
        if (want_mc) {
#pragma unroll
          for (int j = 0; j < Q; ++j) a.marginals_mc[dsc.marg_off + (size_t)m * M + kIt * Q + j] = (float)cnt[j] / (float)C;
        }
      }
    }
  }

  if (a.llrs) {
#pragma unroll
    for (int q = 0; q < kLlrPerThread; ++q) {
      const int it = tid + q * nth;
      if (it < n_llr) {
        R v;
        const R clip = (R)a.llr_clip;
        if (mode == 0) {
          v = lnum[q].value() - lden[q].value();
        } else if (mode == 1) {
          const bool hp = lnum[q].mx > R(-INFINITY), hm = lden[q].mx > R(-INFINITY);
          v = !hp ? -clip : (!hm ? clip : lnum[q].value() - lden[q].value());
          v = v > clip ? clip : (v < -clip ? -clip : v);
        } else {
          const int cm_ = C - cplus[q];
          v = cm_ == 0 ? clip : (cplus[q] == 0 ? -clip : flog(R(cplus[q])) - flog(R(cm_)));
          v = v > clip ? clip : (v < -clip ? -clip : v);
        }
        a.llrs[dsc.llr_off + it] = (float)v;
      }
    }
  }
  // hard decision: smallest recomputed energy among the chains' best states (best_c and
  // best_e were last written before a barrier inside the chunk loop)
  {
    const int bc = best_c;
    if (a.best_energy && tid == 0) a.best_energy[dsc.orig] = (float)best_e;
    if (a.symbols)
      for (int m = tid; m < nt; m += nth)
        a.symbols[dsc.sym_off + m] = Kb[(size_t)bc * Npad + 2 * m] * Q + Kb[(size_t)bc * Npad + 2 * m + 1];
  }
}

// Direct launch (PERS false): instance blockIdx.x.  Persistent launch: items from the list, each
// with its class's arguments.
template <typename R, int Q, bool SH, int BS, bool PERS = false>
__global__ __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(BS == 256 && sizeof(R) == 4 && Q <= 8 ? 5 : 1)))
void estimate_kernel(EstArgs a, Persist p) {
  if constexpr (!PERS) {
    estimate_body<R, Q, SH, BS>(a, blockIdx.x);
  } else {
    extern __shared__ __attribute__((aligned(16))) unsigned char esm[];
    for (;;) {
      const int it = persist_take(p, esm);
      if (it >= p.n_items) break;
      const WorkItem w = p.items[it];
      const EstArgs ca = ((const EstArgs*)p.cls)[__builtin_amdgcn_readfirstlane(w.cls)];
      estimate_body<R, Q, SH, BS>(ca, __builtin_amdgcn_readfirstlane(w.inst));
    }
    persist_done(p);
  }
}

size_t estimate_lds_bytes(int nt, int nr, int M, int N, int chunk, bool fp64) {
  const size_t R = fp64 ? 8 : 4;
  const size_t cm = fp64 ? 32 : 20;
  return cm * (size_t)chunk * nt + R * (3 * (size_t)chunk * nr + 4 * (size_t)chunk + nt + 2 * (size_t)nr) +
         2 * (size_t)chunk * N + 16;
}

// Chains per chunk (LDS budget 96 KiB).  When the (antenna, kI) rows outnumber
// the 256 threads and there are several chunks, the chunks are staged again
// for every block of rows.
// H is staged in LDS when it fits 64 KiB (transposed, padded rows).
static bool estimate_h_in_lds(int nt, int nr, bool fp64) {
  return 2 * (size_t)(nt + 1) * nr * (fp64 ? 8 : 4) <= 65536;
}

// Threads per workgroup: one (antenna, kI) row each, in 256, 512 or 1024 threads; 1024 whenever H is
// read from global memory (the residual and H^H r sweeps, O(C nt nr), then dominate).  The float64
// path (nt <= 32) keeps 256.
static int estimate_threads(int nt, int nr, int Q, bool fp64) {
  if (fp64) return 256;
  if (!estimate_h_in_lds(nt, nr, false) || nt * Q > 512) return 1024;
  return nt * Q > 256 ? 512 : 256;
}

int estimate_chunk(int nt, int nr, int M, int N, int C, bool fp64) {
  int ch = C;
  while (ch > 1 && estimate_lds_bytes(nt, nr, M, N, ch, fp64) > 96 * 1024) ch = (ch + 1) / 2;
  // 256-thread workgroups run five per CU when their LDS (with H staged) fits 32 KiB, 512-thread
  // ones two per CU within 80 KiB: take the smaller chunk that gets there, if it keeps at least
  // 16 chains
  const int Q = M <= 4 ? 2 : (M <= 16 ? 4 : (M <= 64 ? 8 : 16));
  const int bs = estimate_threads(nt, nr, Q, fp64);
  if (!fp64 && bs <= 512) {
    const size_t budget = (bs == 256 ? 32 : 80) * 1024;
    const size_t hx = 2 * (size_t)(nt + 1) * nr * sizeof(float) + 16;   // H is in LDS (bs < 1024)
    int c2 = ch;
    while (c2 > 16 && estimate_lds_bytes(nt, nr, M, N, c2, false) + hx > budget) c2 = (c2 + 1) / 2;
    if (estimate_lds_bytes(nt, nr, M, N, c2, false) + hx <= budget) ch = c2;
  }
  return ch;
}

template <typename R, int Q, int BS>
static hipError_t launch_eb(const EstArgs& a, hipStream_t s, const Persist* p, int gn, KernelCfg* cfg) {
  const size_t hbytes = 2 * (size_t)(a.nt + 1) * a.nr * sizeof(R);
  const bool sh = estimate_h_in_lds(a.nt, a.nr, sizeof(R) == 8);
  const size_t lds = estimate_lds_bytes(a.nt, a.nr, Q * Q, a.N, a.chunk, a.fp64) + (sh ? hbytes + 16 : 0);
  void (*k)(EstArgs, Persist);
  if (p || cfg) k = sh ? estimate_kernel<R, Q, true, BS, true> : estimate_kernel<R, Q, false, BS, true>;
  else k = sh ? estimate_kernel<R, Q, true, BS> : estimate_kernel<R, Q, false, BS>;
  if (cfg) {
    cfg->k = (const void*)k;
    cfg->threads = BS;
    cfg->lds = lds;
    cfg->gx = a.n_inst;
    cfg->gy = 1;
    return hipSuccess;
  }
  // a persistent launch keeps one more aligned word after the body's LDS (the item broadcast)
  const size_t lds_run = p ? ((p->lds_off + 4 + 15) & ~(size_t)15) : lds;
  if (lds_run > 65536) {
    const hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_run);
    if (e != hipSuccess) return e;
  }
  if (p) hipLaunchKernelGGL(k, dim3(gn), dim3(BS), lds_run, s, a, *p);
  else hipLaunchKernelGGL(k, dim3(a.n_inst), dim3(BS), lds, s, a, Persist{});
  return hipGetLastError();
}

template <typename R, int Q>
static hipError_t launch_e(const EstArgs& a, hipStream_t s, const Persist* p, int gn, KernelCfg* cfg) {
  if constexpr (sizeof(R) == 8) {
    return launch_eb<R, Q, 256>(a, s, p, gn, cfg);
  } else {
    const int bs = estimate_threads(a.nt, a.nr, Q, false);
    return bs == 256 ? launch_eb<R, Q, 256>(a, s, p, gn, cfg)
                     : (bs == 512 ? launch_eb<R, Q, 512>(a, s, p, gn, cfg) : launch_eb<R, Q, 1024>(a, s, p, gn, cfg));
  }
}

template <typename R>
static hipError_t launch_r(const EstArgs& a, hipStream_t s, const Persist* p, int gn, KernelCfg* cfg) {
  switch (a.Q) {
    case 2: return launch_e<R, 2>(a, s, p, gn, cfg);
    case 4: return launch_e<R, 4>(a, s, p, gn, cfg);
    case 8: return launch_e<R, 8>(a, s, p, gn, cfg);
    case 16: return launch_e<R, 16>(a, s, p, gn, cfg);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_estimate(const EstArgs& a, hipStream_t s, const Persist* p, int gn, KernelCfg* cfg) {
  return a.fp64 ? launch_r<double>(a, s, p, gn, cfg) : launch_r<float>(a, s, p, gn, cfg);
}

}  // namespace dmala
