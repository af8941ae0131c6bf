// Estimators on the final samples (Algorithm 2, steps after sampling).
//
// One workgroup per instance.  For every chain's final state x^[s] (the sample
// list of Section V-A) the kernel recomputes the residual r = y - H x from the
// inputs, E = ||r||^2, f = -E/sigma^2 and c = H^H r.  A single-coordinate change
// of dimension n by d then has the closed form
//     f(x + d e_n) = f + (2 d c_n - d^2 ||h_m||^2) / sigma^2,
// which gives, per bit (eq. llr_is in the log-sum-exp form of eq. llr_simple,
// F(a) = log(1 + e^a) evaluated exactly)
//     L = LSE_s[((tau-1)/tau) F+ - F(-g)] - LSE_s[((tau-1)/tau) F- - F(g)],  g = (F+ - F-)/tau,
// and per antenna and point a the symbol-level IS estimate
//     p(a) propto sum_s pi_a(a | x^[s]_-m) exp(((tau-1)/tau) f(x^[s]_{m<-a})),
// whose I/Q parts separate because the real-equivalent columns of one antenna
// are orthogonal.  The hard decision is the chain whose tracked best state has
// the smallest freshly recomputed residual energy.
//
// Chains are processed in chunks staged in LDS; every (bit) and (antenna,
// point) output keeps a running log-sum-exp in registers across chunks.
#include "common.hpp"

namespace dmala {

template <typename R>
struct OnlineLse {
  R mx, sum;
  __device__ OnlineLse() : mx(-INFINITY), sum(R(0)) {}
  __device__ void add(R v) {
    if (v == R(-INFINITY)) return;
    if (v > mx) { sum = sum * exp(mx - v) + R(1); mx = v; }
    else sum += exp(v - mx);
  }
  __device__ R value() const { return mx + log(sum); }
};

template <typename R>
__device__ __forceinline__ R softplus(R a) {  // log(1 + e^a)
  return a > R(0) ? a + log1p(exp(-a)) : log1p(exp(a));
}

__device__ __forceinline__ int ungray(int g) {
  g ^= g >> 1; g ^= g >> 2; g ^= g >> 4;
  return g;
}

constexpr int kMaxLlrPerThread = 2;    // nt * log2(M) <= 64 * 8 = 512 = 2 * 256
constexpr int kMaxMargPerThread = 64;  // nt * M <= 64 * 256 = 16384 = 64 * 256

template <typename R, int MPT>
__global__ __launch_bounds__(256) void estimate_kernel(EstArgs a) {
  const int b = blockIdx.x, tid = threadIdx.x, nth = blockDim.x;
  const int nt = a.nt, nr = a.nr, Q = a.Q, M = Q * Q, C = a.C, Npad = a.Npad, N = a.N, CH = a.chunk;
  int nb = 0;
  while ((1 << nb) < Q) ++nb;
  const R* H = (const R*)a.H + 2 * (size_t)b * nt * nr;
  const R* y = (const R*)a.y + 2 * (size_t)b * nr;
  const InstParams ip = *(const InstParams*)(a.ws_inst + (size_t)b * a.inst_stride);
  const R sigma2 = (R)ip.sigma2, s = (R)ip.s, tau = (R)ip.tau;
  const R cw = (tau - R(1)) / tau;
  const StateOff so = state_offsets(a.Cpad, Npad);
  const unsigned char* st = a.ws_state + (size_t)b * a.state_stride;
  const int8_t* K = (const int8_t*)(st + so.k);
  const int8_t* Kb = (const int8_t*)(st + so.kbest);

  extern __shared__ __attribute__((aligned(16))) unsigned char esm[];
  R* rs = (R*)esm;                          // CH x nr complex residuals of the final states
  R* rb2 = rs + 2 * (size_t)CH * nr;        // CH x nr |residual|^2 of the best states
  R* cc = rb2 + (size_t)CH * nr;            // CH x nt complex H^H r
  R* lse = cc + 2 * (size_t)CH * nt;        // CH x nt x 2 per-axis log normalisers
  R* fs = lse + 2 * (size_t)CH * nt;        // CH
  R* ebs = fs + CH;                         // CH
  R* Gd = ebs + CH;                         // nt
  R* lp = Gd + nt;                          // nt x M
  int8_t* Ks = (int8_t*)(lp + (size_t)nt * M);  // CH x N
  int8_t* Kbs = Ks + (size_t)CH * N;            // CH x N
  __shared__ R best_e;
  __shared__ int best_c;

  auto level = [&](int k) { return s * R(2 * k - Q + 1); };

  for (int m = tid; m < nt; m += nth) {
    R g = 0;
    for (int i = 0; i < nr; ++i) {
      const R hre = H[2 * ((size_t)m * nr + i)], him = H[2 * ((size_t)m * nr + i) + 1];
      g += hre * hre + him * him;
    }
    Gd[m] = g;
  }
  if (tid == 0) { best_e = R(INFINITY); best_c = 0; }

  // per-thread accumulators
  const int n_llr = nt * 2 * nb, n_marg = nt * M;
  OnlineLse<R> lnum[kMaxLlrPerThread], lden[kMaxLlrPerThread];
  OnlineLse<R> lmarg[MPT];
  int mc[MPT];
#pragma unroll
  for (int q = 0; q < MPT; ++q) mc[q] = 0;

  for (int c0 = 0; c0 < C; c0 += CH) {
    const int ch = C - c0 < CH ? C - c0 : CH;
    __syncthreads();
    for (int it = tid; it < ch * N; it += nth) {
      const int c = it / N, n = it % N;
      Ks[it] = K[(size_t)(c0 + c) * Npad + n];
      Kbs[it] = Kb[(size_t)(c0 + c) * Npad + n];
    }
    __syncthreads();
    // residuals of the final and of the best states
    for (int it = tid; it < ch * nr; it += nth) {
      const int c = it / nr, i = it % nr;
      R re = y[2 * i], im = y[2 * i + 1];
      R bre = re, bim = im;
      for (int m = 0; m < nt; ++m) {
        const R hre = H[2 * ((size_t)m * nr + i)], him = H[2 * ((size_t)m * nr + i) + 1];
        const R xr = level(Ks[c * N + 2 * m]), xi = level(Ks[c * N + 2 * m + 1]);
        re -= hre * xr - him * xi;
        im -= hre * xi + him * xr;
        const R br = level(Kbs[c * N + 2 * m]), bi = level(Kbs[c * N + 2 * m + 1]);
        bre -= hre * br - him * bi;
        bim -= hre * bi + him * br;
      }
      rs[2 * it] = re;
      rs[2 * it + 1] = im;
      rb2[it] = bre * bre + bim * bim;
    }
    __syncthreads();
    for (int it = tid; it < ch * nt; it += nth) {
      const int c = it / nt, m = it % nt;
      R re = 0, im = 0;
      for (int i = 0; i < nr; ++i) {
        const R hre = H[2 * ((size_t)m * nr + i)], him = H[2 * ((size_t)m * nr + i) + 1];
        const R rr = rs[2 * (c * nr + i)], ri = rs[2 * (c * nr + i) + 1];
        re += hre * rr + him * ri;
        im += hre * ri - him * rr;
      }
      cc[2 * it] = re;
      cc[2 * it + 1] = im;
    }
    for (int c = tid; c < ch; c += nth) {
      R e = 0, eb = 0;
      for (int i = 0; i < nr; ++i) {
        e += rs[2 * (c * nr + i)] * rs[2 * (c * nr + i)] + rs[2 * (c * nr + i) + 1] * rs[2 * (c * nr + i) + 1];
        eb += rb2[c * nr + i];
      }
      fs[c] = -e / sigma2;
      ebs[c] = eb;
    }
    __syncthreads();

    // change of f when coordinate n of sample c moves to level k
    auto delta = [&](int c, int n, int k) {
      const int m = n >> 1;
      const R d = level(k) - level(Ks[c * N + n]);
      return (R(2) * d * cc[2 * (c * nt + m) + (n & 1)] - d * d * Gd[m]) / sigma2;
    };

    for (int it = tid; it < ch * nt; it += nth) {
      const int c = it / nt, m = it % nt;
      for (int ax = 0; ax < 2; ++ax) {
        OnlineLse<R> l;
        for (int k = 0; k < Q; ++k) l.add(delta(c, 2 * m + ax, k) / tau);
        lse[2 * it + ax] = l.value();
      }
    }
    if (tid == 0) {
      for (int c = 0; c < ch; ++c)
        if (ebs[c] < best_e) { best_e = ebs[c]; best_c = c0 + c; }
    }
    __syncthreads();

    // bit LLRs
#pragma unroll
    for (int q = 0; q < kMaxLlrPerThread; ++q) {
      const int it = tid + q * nth;
      if (it < n_llr) {
        const int m = it / (2 * nb), ax = (it / nb) % 2, bit = it % nb;
        const int n = 2 * m + ax;
        const int mask = 1 << (nb - 1 - bit);
        for (int c = 0; c < ch; ++c) {
          const int k = Ks[c * N + n];
          const int g = k ^ (k >> 1);
          const R Fp = fs[c] + delta(c, n, ungray(g & ~mask));
          const R Fm = fs[c] + delta(c, n, ungray(g | mask));
          const R gm = (Fp - Fm) / tau;
          lnum[q].add(cw * Fp - softplus(-gm));
          lden[q].add(cw * Fm - softplus(gm));
        }
      }
    }
    // symbol marginals (IS) and the plain Monte Carlo histogram
#pragma unroll
    for (int q = 0; q < MPT; ++q) {
      const int it = tid + q * nth;
      if (it < n_marg) {
        const int m = it / M, pt = it % M, kI = pt / Q, kQ = pt % Q;
        for (int c = 0; c < ch; ++c) {
          const R v = cw * fs[c] + delta(c, 2 * m, kI) + delta(c, 2 * m + 1, kQ)
                      - lse[2 * (c * nt + m)] - lse[2 * (c * nt + m) + 1];
          lmarg[q].add(v);
          mc[q] += (Ks[c * N + 2 * m] == kI && Ks[c * N + 2 * m + 1] == kQ) ? 1 : 0;
        }
      }
    }
  }

  if (a.llrs) {
#pragma unroll
    for (int q = 0; q < kMaxLlrPerThread; ++q) {
      const int it = tid + q * nth;
      if (it < n_llr) a.llrs[(size_t)b * n_llr + it] = (float)(lnum[q].value() - lden[q].value());
    }
  }
#pragma unroll
  for (int q = 0; q < MPT; ++q) {
    const int it = tid + q * nth;
    if (it < n_marg) {
      lp[it] = lmarg[q].value();
      if (a.marginals_mc) a.marginals_mc[(size_t)b * n_marg + it] = (float)mc[q] / (float)C;
    }
  }
  __syncthreads();
  if (a.marginals) {
    for (int m = tid; m < nt; m += nth) {
      OnlineLse<R> l;
      for (int pt = 0; pt < M; ++pt) l.add(lp[(size_t)m * M + pt]);
      const R z = l.value();
      for (int pt = 0; pt < M; ++pt) a.marginals[((size_t)b * nt + m) * M + pt] = (float)exp(lp[(size_t)m * M + pt] - z);
    }
  }
  // hard decision: smallest recomputed energy among the chains' best states
  if (tid == 0) {
    const int bc = best_c;
    if (a.best_energy) a.best_energy[b] = (float)best_e;
    if (a.symbols)
      for (int m = 0; m < nt; ++m)
        a.symbols[(size_t)b * nt + m] = Kb[(size_t)bc * Npad + 2 * m] * Q + Kb[(size_t)bc * Npad + 2 * m + 1];
  }
}

size_t estimate_lds_bytes(int nt, int nr, int M, int N, int chunk, bool fp64) {
  const size_t R = fp64 ? 8 : 4;
  return R * (3 * (size_t)chunk * nr + 4 * (size_t)chunk * nt + 2 * (size_t)chunk + nt + (size_t)nt * M) +
         2 * (size_t)chunk * N + 16;
}

int estimate_chunk(int nt, int nr, int M, int N, int C, bool fp64) {
  int ch = C;
  while (ch > 1 && estimate_lds_bytes(nt, nr, M, N, ch, fp64) > 96 * 1024) ch = (ch + 1) / 2;
  return ch;
}

template <typename R, int MPT>
static hipError_t launch_e(const EstArgs& a, hipStream_t s) {
  const size_t lds = estimate_lds_bytes(a.nt, a.nr, a.Q * a.Q, a.N, a.chunk, a.fp64);
  auto k = estimate_kernel<R, MPT>;
  if (lds > 65536) {
    const hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k, dim3(a.n_inst), dim3(256), lds, s, a);
  return hipGetLastError();
}

template <typename R>
static hipError_t launch_r(const EstArgs& a, hipStream_t s) {
  const int items = a.nt * a.Q * a.Q;
  if (items <= 256) return launch_e<R, 1>(a, s);
  if (items <= 2048) return launch_e<R, 8>(a, s);
  if (items <= 4096) return launch_e<R, 16>(a, s);
  if (items <= 8192) return launch_e<R, 32>(a, s);
  return launch_e<R, kMaxMargPerThread>(a, s);
}

hipError_t launch_estimate(const EstArgs& a, hipStream_t s) {
  return a.fp64 ? launch_r<double>(a, s) : launch_r<float>(a, s);
}

}  // namespace dmala
