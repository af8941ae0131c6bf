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

template <typename R, typename TIn>
__global__ __launch_bounds__(256) void estimate_kernel(EstArgs a) {
  const int b = blockIdx.x, tid = threadIdx.x, nth = blockDim.x;
  const int nt = a.nt, nr = a.nr, Q = a.Q, M = Q * Q, C = a.C, Npad = a.Npad;
  int nb = 0;
  while ((1 << nb) < Q) ++nb;
  const TIn* H = (const TIn*)a.H + 2 * (size_t)b * nt * nr;
  const TIn* y = (const TIn*)a.y + 2 * (size_t)b * nr;
  const InstParams ip = *(const InstParams*)(a.ws_inst + (size_t)b * a.inst_stride);
  const R sigma2 = (R)ip.sigma2, s = (R)ip.s, tau = (R)ip.tau;
  const R cw = (tau - R(1)) / tau;
  const StateOff so = state_offsets(a.Cpad, Npad);
  const unsigned char* st = a.ws_state + (size_t)b * a.state_stride;
  const int8_t* K = (const int8_t*)(st + so.k);
  const int8_t* Kb = (const int8_t*)(st + so.kbest);

  R* r = (R*)(a.ws_est + (size_t)b * a.est_stride);       // C x nr complex
  R* rb2 = r + 2 * (size_t)C * nr;                           // C x nr
  R* cc = rb2 + (size_t)C * nr;                              // C x nt complex
  R* f = cc + 2 * (size_t)C * nt;                            // C
  R* Efr = f + C;                                            // C
  R* lse = Efr + C;                                          // C x nt x 2
  R* Gd = lse + 2 * (size_t)C * nt;                          // nt
  R* lp = Gd + nt;                                           // nt x M

  auto level = [&](int k) { return s * R(2 * k - Q + 1); };

  // residuals of the final and of the best states
  for (int it = tid; it < C * nr; it += nth) {
    const int c = it / nr, i = it % nr;
    R re = (R)y[2 * i], im = (R)y[2 * i + 1];
    R bre = re, bim = im;
    for (int m = 0; m < nt; ++m) {
      const R hre = (R)H[2 * ((size_t)m * nr + i)], him = (R)H[2 * ((size_t)m * nr + i) + 1];
      const R xr = level(K[(size_t)c * Npad + 2 * m]), xi = level(K[(size_t)c * Npad + 2 * m + 1]);
      re -= hre * xr - him * xi;
      im -= hre * xi + him * xr;
      const R br = level(Kb[(size_t)c * Npad + 2 * m]), bi = level(Kb[(size_t)c * Npad + 2 * m + 1]);
      bre -= hre * br - him * bi;
      bim -= hre * bi + him * br;
    }
    r[2 * (size_t)it] = re;
    r[2 * (size_t)it + 1] = im;
    rb2[it] = bre * bre + bim * bim;
  }
  __syncthreads();
  for (int it = tid; it < C * nt; it += nth) {
    const int c = it / nt, m = it % nt;
    R re = 0, im = 0;
    for (int i = 0; i < nr; ++i) {
      const R hre = (R)H[2 * ((size_t)m * nr + i)], him = (R)H[2 * ((size_t)m * nr + i) + 1];
      const R rr = r[2 * ((size_t)c * nr + i)], ri = r[2 * ((size_t)c * nr + i) + 1];
      re += hre * rr + him * ri;
      im += hre * ri - him * rr;
    }
    cc[2 * (size_t)it] = re;
    cc[2 * (size_t)it + 1] = im;
  }
  for (int c = tid; c < C; c += nth) {
    R e = 0, eb = 0;
    for (int i = 0; i < nr; ++i) {
      e += r[2 * ((size_t)c * nr + i)] * r[2 * ((size_t)c * nr + i)] + r[2 * ((size_t)c * nr + i) + 1] * r[2 * ((size_t)c * nr + i) + 1];
      eb += rb2[(size_t)c * nr + i];
    }
    f[c] = -e / sigma2;
    Efr[c] = eb;
  }
  for (int m = tid; m < nt; m += nth) {
    R g = 0;
    for (int i = 0; i < nr; ++i) {
      const R hre = (R)H[2 * ((size_t)m * nr + i)], him = (R)H[2 * ((size_t)m * nr + i) + 1];
      g += hre * hre + him * him;
    }
    Gd[m] = g;
  }
  __syncthreads();

  // change of f when coordinate n of sample c moves to level k
  auto delta = [&](int c, int n, int k) {
    const int m = n >> 1;
    const R d = level(k) - level(K[(size_t)c * Npad + n]);
    return (R(2) * d * cc[2 * ((size_t)c * nt + m) + (n & 1)] - d * d * Gd[m]) / sigma2;
  };

  // per-sample log normalisers of the tempered conditional of each axis
  for (int it = tid; it < C * nt; it += nth) {
    const int c = it / nt, m = it % nt;
    for (int ax = 0; ax < 2; ++ax) {
      OnlineLse<R> l;
      for (int k = 0; k < Q; ++k) l.add(delta(c, 2 * m + ax, k) / tau);
      lse[2 * (size_t)it + ax] = l.value();
    }
  }
  __syncthreads();

  // bit LLRs
  if (a.llrs) {
    for (int it = tid; it < nt * 2 * nb; it += nth) {
      const int m = it / (2 * nb), ax = (it / nb) % 2, bit = it % nb;
      const int n = 2 * m + ax;
      const int mask = 1 << (nb - 1 - bit);
      OnlineLse<R> num, den;
      for (int c = 0; c < C; ++c) {
        const int k = K[(size_t)c * Npad + n];
        const int g = k ^ (k >> 1);
        const R Fp = f[c] + delta(c, n, ungray(g & ~mask));
        const R Fm = f[c] + delta(c, n, ungray(g | mask));
        const R gm = (Fp - Fm) / tau;
        num.add(cw * Fp - softplus(-gm));
        den.add(cw * Fm - softplus(gm));
      }
      a.llrs[(size_t)b * nt * 2 * nb + it] = (float)(num.value() - den.value());
    }
  }

  // symbol marginals
  if (a.marginals) {
    for (int it = tid; it < nt * M; it += nth) {
      const int m = it / M, pt = it % M, kI = pt / Q, kQ = pt % Q;
      OnlineLse<R> l;
      for (int c = 0; c < C; ++c) {
        const R v = cw * f[c] + delta(c, 2 * m, kI) + delta(c, 2 * m + 1, kQ)
                    - lse[2 * ((size_t)c * nt + m)] - lse[2 * ((size_t)c * nt + m) + 1];
        l.add(v);
      }
      lp[it] = l.value();
    }
    __syncthreads();
    for (int m = tid; m < nt; m += nth) {
      OnlineLse<R> l;
      for (int pt = 0; pt < M; ++pt) l.add(lp[(size_t)m * M + pt]);
      const R z = l.value();
      for (int pt = 0; pt < M; ++pt) a.marginals[((size_t)b * nt + m) * M + pt] = (float)exp(lp[(size_t)m * M + pt] - z);
    }
  }

  if (a.marginals_mc) {
    for (int it = tid; it < nt * M; it += nth) {
      const int m = it / M, pt = it % M;
      int cnt = 0;
      for (int c = 0; c < C; ++c) cnt += (K[(size_t)c * Npad + 2 * m] * Q + K[(size_t)c * Npad + 2 * m + 1]) == pt;
      a.marginals_mc[(size_t)b * nt * M + it] = (float)cnt / (float)C;
    }
  }

  // hard decision: smallest recomputed energy among the chains' best states
  if (tid == 0) {
    int best = 0;
    for (int c = 1; c < C; ++c)
      if (Efr[c] < Efr[best]) best = c;
    if (a.best_energy) a.best_energy[b] = (float)Efr[best];
    if (a.symbols)
      for (int m = 0; m < nt; ++m)
        a.symbols[(size_t)b * nt + m] = Kb[(size_t)best * Npad + 2 * m] * Q + Kb[(size_t)best * Npad + 2 * m + 1];
  }
}

hipError_t launch_estimate(const EstArgs& a, hipStream_t s) {
  if (a.fp64)
    hipLaunchKernelGGL((estimate_kernel<double, double>), dim3(a.n_inst), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL((estimate_kernel<float, float>), dim3(a.n_inst), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace dmala
