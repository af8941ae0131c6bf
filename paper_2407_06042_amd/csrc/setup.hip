// Instance setup: Gram matrix, matched filter, preconditioner and packing.
//
// One workgroup per instance, float64 arithmetic.  Computes in the complex
// form (the real-equivalent matrices of eq. sys_model are expanded only when
// packing):
//   G = H^H H, z = H^H y, ||y||^2                      (gradient of eq. grad: grad f = -(2/sigma^2)(Gx - z))
//   M = (G + gamma I)^-1 by in-place Gauss-Jordan       (preconditioner of the Remark after Algorithm 1;
//                                                         G + gamma I is Hermitian positive definite, so no pivoting)
//   A = M G = I - gamma M,  b = M z                     (so that M grad f = -(2/sigma^2)(A x - b))
// and writes, scaled to the index units of the sampler (see common.hpp),
//   energy matrix  EG = 2 s^2 log2(e)/(tau sigma^2) * R(G),  ez = 2 s log2(e)/(tau sigma^2) * R(z)
//   proposal matrix P = alpha/(2 tau sigma^2) * R(A),       pb = alpha/(2 tau sigma^2 s) * R(b)
// where R(.) is the Re/Im-interleaved real-equivalent.  The MFMA path also
// stores two per-antenna features of the learned proposal's network, in index
// units (level step 2 s): af_{2m} = log2(sigma^2 M_mm / (8 s^2)) / 8 (variance
// of the damped LS estimate) and af_{2m+1} = log2(sigma^2 / (8 s^2 G_mm)) / 8
// (variance of one axis given the others).  On the MFMA path each
// matrix is scaled by a power of two and split into fp16 (or bf16) terms laid
// out as 16x16x32 MFMA A-operand fragments; on the float64 path it is stored
// as a dense row-major array.
#include "common.hpp"

namespace dmala {

struct cd { double re, im; };
__device__ __forceinline__ cd cadd(cd a, cd b) { return {a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ cd cmul(cd a, cd b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ __forceinline__ cd cconjmul(cd a, cd b) { return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re}; }

// Entry (n, n2) of the interleaved real-equivalent of complex X (leading dimension ld).
__device__ __forceinline__ double realeq(const cd* X, int ld, int n, int n2) {
  const cd v = X[(n >> 1) * ld + (n2 >> 1)];
  const int a = n & 1, b = n2 & 1;
  return (a == b) ? v.re : (a == 0 ? -v.im : v.im);
}
__device__ __forceinline__ double realeq_vec(const cd* v, int n) { return (n & 1) ? v[n >> 1].im : v[n >> 1].re; }

// Value of v in lane `lane` of the wavefront (lane uniform).
__device__ __forceinline__ double readlane_f64(double v, int lane) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, lane);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), lane);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Four complex entries 16 TPR bytes apart from LDS address a, waited for in
// the same block: the Gauss-Jordan update keeps four row entries in flight
// (the compiler would otherwise load all of them at once and spill the matrix).
typedef double d2v __attribute__((ext_vector_type(2)));
template <int TPR>
__device__ __forceinline__ void lds_read4(uint32_t a, d2v (&r)[4]) {
  asm volatile(
      "ds_read2_b64 %0, %4 offset1:1\n\t"
      "ds_read2_b64 %1, %4 offset0:%5 offset1:%6\n\t"
      "ds_read2_b64 %2, %4 offset0:%7 offset1:%8\n\t"
      "ds_read2_b64 %3, %4 offset0:%9 offset1:%10\n\t"
      "s_waitcnt lgkmcnt(0)"
      : "=&v"(r[0]), "=&v"(r[1]), "=&v"(r[2]), "=&v"(r[3])
      : "v"(a), "i"(2 * TPR), "i"(2 * TPR + 1), "i"(4 * TPR), "i"(4 * TPR + 1), "i"(6 * TPR), "i"(6 * TPR + 1)
      : "memory");
}

__device__ double block_reduce(double v, double* red, bool is_max) {
  const int tid = threadIdx.x;
  red[tid] = v;
  __syncthreads();
  for (int w = blockDim.x >> 1; w > 0; w >>= 1) {
    if (tid < w) red[tid] = is_max ? fmax(red[tid], red[tid + w]) : red[tid] + red[tid + w];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

// double -> float in hardware, kept as a separate step: the compiler would otherwise
// fold the two conversions to half (or bfloat16) into one emulated in software.
__device__ __forceinline__ float via_float(double v) {
  float f = (float)v;
  asm volatile("" : "+v"(f));
  return f;
}

// Pack c * R(X) (N x N, zero-padded to Npad) into MFMA fragments.
// npass = 3 (fp16 lo, mid, hi), 2 (fp16 lo, hi) or 1 (fp16 or bf16 when bf16 != 0);
// the terms are stored in accumulation order, small terms first.
// Fragment (pass p, row tile rt, K block kb) lane l element j holds entry
// (16 rt + l%16, 16 (2 kb + j/4) + 4 (l/16) + j%4): the K order matches the
// dimensions each lane owns in the accumulator layout, so the sampler builds
// the B operand from its own registers.
// With cx != 0 the complex planes are packed instead (the sampler's complex-plane layouts): pass p,
// plane pl (real, imaginary), antenna tile at (16 rows), K block kb of 32 antennas; lane l element j
// holds plane(X)[16 at + l%16][16 (2 kb + j/4) + 4 (l/16) + j%4] -- the same K permutation over
// antennas that the real-equivalent packing applies to real dimensions.
__device__ float pack_fragments(const cd* X, int ld, double c, int nt, int N, int RT, int KB, int npass, int bf16,
                                unsigned char* dst, double* red, int cx) {
  double mx = 0.0;
  for (int e = threadIdx.x; e < nt * nt; e += blockDim.x) {
    const cd v = X[(e / nt) * ld + e % nt];
    mx = fmax(mx, fmax(fabs(v.re), fabs(v.im)));
  }
  mx = block_reduce(mx, red, true) * fabs(c);
  int ex = 0;
  if (mx > 0.0) frexp(mx, &ex);
  const int e2 = 14 - ex;  // scaled max in [2^13, 2^14)
  const double sc = ldexp(c, e2);
  const int AT = RT / 2, KBX = RT / 4;
  const size_t pass_stride = cx ? (size_t)2 * AT * KBX * 1024 : (size_t)RT * KB * 1024;
  const int items = (int)(pass_stride / 16);
  for (int it = threadIdx.x; it < items; it += blockDim.x) {
    const int l = it & 63;
    const int t = it >> 6;
    // real-equivalent: (row tile, K block); complex planes: (plane, antenna tile, K block)
    const int kb = cx ? t % KBX : t % KB;
    const int rt = cx ? (t / KBX) % AT : t / KB;
    const int pl = cx ? t / (KBX * AT) : 0;
    const int n = 16 * rt + (l & 15);
    union { _Float16 h[8]; __bf16 b[8]; uint4 u; } f0, f1, f2;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int n2 = 16 * (2 * kb + (j >> 2)) + 4 * (l >> 4) + (j & 3);
      double v;
      if (cx) {
        const cd e = X[(n < nt && n2 < nt ? n : 0) * ld + (n2 < nt ? n2 : 0)];
        v = (n < nt && n2 < nt) ? sc * (pl ? e.im : e.re) : 0.0;
      } else {
        v = (n < N && n2 < N) ? sc * realeq(X, ld, n, n2) : 0.0;
      }
      if (bf16) {
        f0.b[j] = (__bf16)via_float(v);
      } else {
        const _Float16 hi = (_Float16)via_float(v);
        const double r1 = v - (double)hi;
        const _Float16 mid = (_Float16)via_float(r1);
        const double r2 = r1 - (double)mid;
        if (npass == 3) { f0.h[j] = (_Float16)via_float(r2); f1.h[j] = mid; f2.h[j] = hi; }
        else if (npass == 2) { f0.h[j] = mid; f1.h[j] = hi; }
        else f0.h[j] = hi;
      }
    }
    unsigned char* o = dst + (size_t)t * 1024 + l * 16;
    *(uint4*)o = f0.u;
    if (npass > 1) *(uint4*)(o + pass_stride) = f1.u;
    if (npass > 2) *(uint4*)(o + 2 * pass_stride) = f2.u;
  }
  return (float)ldexp(1.0, -e2);
}

// Dense row-major double copy of c * R(X), zero-padded to Npad x Npad.
__device__ void pack_dense(const cd* X, int ld, double c, int N, int Npad, double* dst) {
  for (int e = threadIdx.x; e < Npad * Npad; e += blockDim.x) {
    const int n = e / Npad, n2 = e % Npad;
    dst[e] = (n < N && n2 < N) ? c * realeq(X, ld, n, n2) : 0.0;
  }
}

// 256-thread workgroups (instances up to 32 antennas) run five per CU: at most 96 registers, and
// about 31 KiB of LDS with H staged 16 receive antennas at a time.
// RMAX: rows of the working matrix the Gauss-Jordan register layout covers (threads per row BS / RMAX).
template <typename TIn, bool WGLOB, int BS, int RMAX>
__global__ __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(BS == 256 ? (WGLOB ? 4 : 5) : 1)))
void setup_kernel(SetupArgs a) {
  const int b = blockIdx.x, tid = threadIdx.x, nt = a.nt, nr = a.nr, N = a.N, Npad = a.Npad;
  const int ld = nt + 1;  // padded leading dimension of the LDS matrices (no bank conflicts on columns)
  const InstDesc dsc = inst_desc(a.desc, b, nt, nr, a.Q * a.Q, 1);
  const TIn* Hg = (const TIn*)a.H + 2 * dsc.h_off;
  const TIn* y = (const TIn*)a.y + 2 * dsc.y_off;
  const double sigma2 = a.sigma2 ? (double)((const TIn*)a.sigma2)[dsc.orig] : a.sigma2_val;
  extern __shared__ double smem_setup[];
  // nt x ld working matrix: in LDS, or (large nt) in this instance's slice of the workspace
  cd* W;
  cd* z;
  if constexpr (WGLOB) {
    W = (cd*)(a.wscratch + (size_t)b * a.wscratch_stride);
    z = (cd*)smem_setup;
  } else {
    W = (cd*)smem_setup;
    z = W + nt * ld;
  }
  cd* bv = z + nt;
  cd* rowp = bv + nt;       // 2 x nt (alternating Gauss-Jordan steps)
  cd* colp = rowp + 2 * nt; // 2 x nt
  double* red = (double*)(colp + 2 * nt);
  unsigned char* blk = a.ws_inst + (size_t)b * a.inst_stride;

  const int Q = a.Q, M = Q * Q;
  const double s = sqrt(3.0 / (2.0 * (M - 1)));
  const double tau = a.tau;
  const double alpha = a.alpha_mult * sigma2;
  const double beta = a.naive ? 1.0 : a.beta_mult * s * s / sigma2;
  const double gamma = a.gamma_mult * sigma2 / (2.0 * s * s);

  // G = H^H H and z = H^H y.  H is staged in LDS in chunks of receive
  // antennas, transposed with a padded row (Ht[i][m]); each thread accumulates
  // its (m, m2) entries (and entries of z) in registers across the chunks.
  double nonfinite = 0.0;
  {
    // H is staged in LDS in chunks of receive antennas, transposed with a padded
    // row whose last entry holds y (Ht[i][m], Ht[i][nt] = y_i), so that z is one
    // more column of the product: z_m = (H^H [H y])_{m, nt}.  Each thread
    // accumulates a 2 x 2 block of entries in registers across the chunks; only
    // blocks on or above the diagonal and the blocks of the z column are
    // computed, and the lower triangle is written as the conjugate.
    constexpr int kIC = BS == 256 ? 16 : 32;
    constexpr int kBPT = WGLOB ? (BS >= 1024 || BS == 256 ? 3 : 2) : 1;  // blocks per thread per group (one group for every nt)
    cd* Ht = (cd*)(red + BS);               // kIC x ld, then one spare row read past the last column
    const int nb = (nt + 1) >> 1;           // 2-row blocks
    const int nbu = nb * (nb + 1) / 2;      // blocks on or above the diagonal
    const int nblk = nbu + nb;              // ... and the z column
    for (int b0 = 0; b0 < nblk; b0 += kBPT * BS) {
      int m[kBPT], m2[kBPT];
      cd acc[kBPT][2][2];
#pragma unroll
      for (int q = 0; q < kBPT; ++q) {
        int bi = b0 + tid + q * BS;
        if (bi < nbu) {           // upper block (br, bc), bc >= br, row-major over the triangle
          int br = 0;
          while (bi >= nb - br) { bi -= nb - br; ++br; }
          m[q] = 2 * br;
          m2[q] = 2 * (br + bi);
        } else {                  // z block (past nblk: idle)
          m[q] = 2 * (bi - nbu);
          m2[q] = nt;
        }
#pragma unroll
        for (int r = 0; r < 2; ++r)
#pragma unroll
          for (int c = 0; c < 2; ++c) acc[q][r][c] = {0.0, 0.0};
      }
      for (int i0 = 0; i0 < nr; i0 += kIC) {
        const int ic = nr - i0 < kIC ? nr - i0 : kIC;
        for (int e = tid; e < ic * (nt + 1); e += BS) {
          const int mm = e / ic, ii = e % ic;
          const TIn* src = mm < nt ? Hg + 2 * ((size_t)mm * nr + i0 + ii) : y + 2 * (i0 + ii);
          Ht[ii * ld + mm] = {(double)src[0], (double)src[1]};
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < kBPT; ++q) {
          if (b0 + tid + q * BS < nblk) {
            // reads reach one entry past a row (column nt + 1, or row nt of an odd nt):
            // those products are never stored
            const cd* ha = Ht + m[q];
            const cd* hb = Ht + m2[q];
            for (int ii = 0; ii < ic; ++ii) {
              const cd a0 = ha[ii * ld], a1 = ha[ii * ld + 1];
              const cd c0 = hb[ii * ld], c1 = hb[ii * ld + 1];
              const cd av[2] = {a0, a1}, cv[2] = {c0, c1};
#pragma unroll
              for (int r = 0; r < 2; ++r)
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                  cd& g = acc[q][r][c];
                  g.re = fma(av[r].re, cv[c].re, fma(av[r].im, cv[c].im, g.re));
                  g.im = fma(av[r].re, cv[c].im, fma(-av[r].im, cv[c].re, g.im));
                }
            }
          }
        }
        __syncthreads();
      }
#pragma unroll
      for (int q = 0; q < kBPT; ++q) {
        if (b0 + tid + q * BS < nblk) {
#pragma unroll
          for (int r = 0; r < 2; ++r)
#pragma unroll
            for (int c = 0; c < 2; ++c) {
              const int i = m[q] + r, j = m2[q] + c;
              const cd g = acc[q][r][c];
              if (i >= nt) continue;
              if (m2[q] == nt) {
                if (c == 0) z[i] = g;
                else continue;
              } else if (j < nt) {
                W[i * ld + j] = g;
                if (m2[q] != m[q]) W[j * ld + i] = {g.re, -g.im};
              } else {
                continue;
              }
              if (!isfinite(g.re) || !isfinite(g.im)) nonfinite = 1.0;
            }
        }
      }
    }
  }
  double yy = 0.0;
  for (int i = tid; i < nr; i += blockDim.x) {
    const double re = (double)y[2 * i], im = (double)y[2 * i + 1];
    yy += re * re + im * im;
  }
  __syncthreads();
  yy = block_reduce(yy, red, false);
  if (!isfinite(yy) || !(sigma2 > 0.0) || !isfinite(sigma2)) nonfinite = 1.0;
  nonfinite = block_reduce(nonfinite, red, true);

  const double cE = 2.0 * s * s * kLog2e / (tau * sigma2);
  const double cz = 2.0 * s * kLog2e / (tau * sigma2);
  const double cP = alpha / (2.0 * tau * sigma2);
  const double cb = alpha / (2.0 * tau * sigma2 * s);
  const int npP = p_passes(a.pm);
  unsigned char* frag = blk + kParamBytes;
  // bytes of one split term of a packed matrix (real-equivalent, or complex planes: half of it)
  const size_t pass_bytes = a.cx ? (size_t)a.RT * a.RT / 4 * 1024 : (size_t)a.RT * a.KB * 1024;
  float scaleE = 1.0f, scaleP = 1.0f;

  // energy matrix and vector
  if (a.fp64) {
    double* EGd = (double*)(blk + kParamBytes) + (size_t)Npad * Npad;
    pack_dense(W, ld, cE, N, Npad, EGd);
    double* ezd = (double*)(blk + kParamBytes) + 2 * (size_t)Npad * Npad + Npad;
    for (int n = tid; n < Npad; n += blockDim.x) ezd[n] = n < N ? cz * realeq_vec(z, n) : 0.0;
  } else {
    scaleE = pack_fragments(W, ld, cE, nt, N, a.RT, a.KB, kEPasses, 0, frag + (size_t)npP * pass_bytes, red, a.cx);
    float* ezf = (float*)(frag + (size_t)(npP + kEPasses) * pass_bytes) + Npad;
    for (int n = tid; n < Npad; n += blockDim.x) ezf[n] = n < N ? (float)(cz * realeq_vec(z, n)) : 0.0f;
    float* afv = ezf + Npad;
    for (int n = tid; n < Npad; n += blockDim.x) {
      const int m = n >> 1;
      afv[n] = (n < N && (n & 1)) ? (float)(log2(sigma2 / (8.0 * s * s * W[m * ld + m].re)) / 8.0) : 0.0f;
    }
  }
  __syncthreads();

  if (!a.naive) {
    // W <- (G + gamma I)^-1 by in-place Gauss-Jordan
    for (int m = tid; m < nt; m += blockDim.x) W[m * ld + m].re += gamma;
    __syncthreads();
    // Gauss-Jordan with the working matrix in registers: thread t keeps row
    // t / TPR, columns t % TPR + TPR k (k < KMAX), for the whole sweep.  A step on
    // pivot p: the owners of column p publish it (colp); the threads of row p,
    // which share a wavefront with the pivot, read the pivot from its lane, scale
    // their row by its inverse (the inverse itself in column p) and publish it
    // (rowp); after one barrier every other row i clears its column p and
    // subtracts colp[i] * rowp, which leaves -w_ip / w_pp there.  The steps on
    // different pivots commute (G + gamma I is Hermitian positive definite, so
    // every pivot stays nonzero in any order), so they run in the order
    // p = o + TPR kb, o outer: column p then sits in register slot kb, a
    // compile-time index of the unrolled inner loop.  The two vectors alternate
    // between steps, so one barrier per step orders all reads and writes.
    constexpr int TPR = BS / RMAX;                               // threads per row
    constexpr int KMAX = RMAX / TPR;                             // columns per thread
    static_assert(64 % TPR == 0, "the threads of a row share a wavefront");
    static_assert(KMAX % 4 == 0 && 6 * TPR + 1 < 256, "row entries are read four at a time");
    const int gi = tid / TPR, gj = tid % TPR;
    cd w[KMAX];
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
      const int j = gj + TPR * k;
      w[k] = (gi < nt && j < nt) ? W[gi * ld + j] : cd{0.0, 0.0};
    }
    int par = 0;
#pragma unroll 1
    for (int o = 0; o < TPR && o < nt; ++o) {
#pragma unroll
      for (int kb = 0; kb < KMAX; ++kb) {
        const int p = o + TPR * kb;
        if (p < nt) {
          cd* rp = rowp + par * nt;
          cd* cp = colp + par * nt;
          par ^= 1;
          if (gi < nt && gj == o) cp[gi] = w[kb];
          if (gi == p) {
            const int lane = (p * TPR + o) & 63;
            const cd piv = {readlane_f64(w[kb].re, lane), readlane_f64(w[kb].im, lane)};
            const double rd = 1.0 / (piv.re * piv.re + piv.im * piv.im);
            const cd inv = {piv.re * rd, -piv.im * rd};
#pragma unroll
            for (int k = 0; k < KMAX; ++k) w[k] = cmul(w[k], inv);
            if (gj == o) w[kb] = inv;
#pragma unroll
            for (int k = 0; k < KMAX; ++k) {
              const int j = gj + TPR * k;
              if (j < nt) rp[j] = w[k];
            }
          }
          __syncthreads();
          if (gi < nt && gi != p) {
            const cd ci = cp[gi];
            if (gj == o) w[kb] = {0.0, 0.0};
            // entries past column nt - 1 read whatever follows rowp in LDS (inside the
            // allocation); they are never stored
            const uint32_t ra = (uint32_t)(uintptr_t)(__attribute__((address_space(3))) cd*)(rp + gj);
#pragma unroll
            for (int k0 = 0; k0 < KMAX; k0 += 4) {
              if (TPR * k0 < nt) {
                d2v r[4];
                lds_read4<TPR>(ra + 16 * TPR * k0, r);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                  cd& v = w[k0 + q];
                  v.re = fma(-ci.re, r[q].x, fma(ci.im, r[q].y, v.re));
                  v.im = fma(-ci.re, r[q].y, fma(-ci.im, r[q].x, v.im));
                }
              }
            }
          }
        }
      }
    }
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
      const int j = gj + TPR * k;
      if (gi < nt && j < nt) W[gi * ld + j] = w[k];
    }
    __syncthreads();
    if (!a.fp64) {
      float* afv = (float*)(frag + (size_t)(npP + kEPasses) * pass_bytes) + 2 * Npad;
      for (int m = tid; m < nt; m += blockDim.x)
        afv[2 * m] = (float)(log2(sigma2 * W[m * ld + m].re / (8.0 * s * s)) / 8.0);
    }
    // b = M z, then W <- A = I - gamma M
    for (int m = tid; m < nt; m += blockDim.x) {
      cd acc = {0.0, 0.0};
      for (int j = 0; j < nt; ++j) acc = cadd(acc, cmul(W[m * ld + j], z[j]));
      bv[m] = acc;
    }
    __syncthreads();
    for (int e = tid; e < nt * nt; e += blockDim.x) {
      const int i = e / nt, j = e % nt;
      W[i * ld + j] = {(i == j ? 1.0 : 0.0) - gamma * W[i * ld + j].re, -gamma * W[i * ld + j].im};
    }
    __syncthreads();
    if (a.fp64) {
      pack_dense(W, ld, cP, N, Npad, (double*)(blk + kParamBytes));
      double* pbd = (double*)(blk + kParamBytes) + 2 * (size_t)Npad * Npad;
      for (int n = tid; n < Npad; n += blockDim.x) pbd[n] = n < N ? cb * realeq_vec(bv, n) : 0.0;
    } else {
      scaleP = pack_fragments(W, ld, cP, nt, N, a.RT, a.KB, npP, a.pm == PM_BF16X1, frag, red, a.cx);
      float* pbf = (float*)(frag + (size_t)(npP + kEPasses) * pass_bytes);
      for (int n = tid; n < Npad; n += blockDim.x) pbf[n] = n < N ? (float)(cb * realeq_vec(bv, n)) : 0.0f;
    }
  } else if (a.fp64) {
    double* Pd = (double*)(blk + kParamBytes);
    for (int e = tid; e < Npad * Npad; e += blockDim.x) Pd[e] = 0.0;
    double* pbd = Pd + 2 * (size_t)Npad * Npad;
    for (int n = tid; n < Npad; n += blockDim.x) pbd[n] = 0.0;
  }

  if (tid == 0) {
    InstParams ip;
    ip.yy = yy;
    ip.eunit = tau * sigma2 / kLog2e;
    ip.kL = kLog2e * 2.0 * s * s / (alpha * beta);
    ip.rho = alpha / (4.0 * s * s * kLog2e);
    ip.sigma2 = sigma2;
    ip.s = s;
    ip.tau = tau;
    ip.scaleP = scaleP;
    ip.scaleE = scaleE;
    ip.nonfinite = nonfinite > 0.0 ? 1 : 0;
    ip.pad_[0] = ip.pad_[1] = ip.pad_[2] = 0;
    *(InstParams*)blk = ip;
    if (a.status) a.status[dsc.orig] = ip.nonfinite ? kStatusNonfinite : 0;
  }
}

bool setup_w_global(int nt) { return nt > 32; }

template <int BS, bool WG, int RMAX>
hipError_t launch_setup_bs(const SetupArgs& a, hipStream_t s) {
  if (WG != setup_w_global(a.nt) || a.nt > RMAX) return hipErrorInvalidValue;
  const size_t lds = (size_t)((WG ? 0 : a.nt * (a.nt + 1)) + 6 * a.nt) * sizeof(cd) + BS * sizeof(double) +
                     ((BS == 256 ? 16 : 32) * (size_t)(a.nt + 1) + 32) * sizeof(cd);
  void (*k)(SetupArgs) = a.fp64 ? setup_kernel<double, WG, BS, RMAX> : setup_kernel<float, WG, BS, RMAX>;
  if (lds > 65536) {
    const hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k, dim3(a.n_inst), dim3(BS), lds, s, a);
  return hipGetLastError();
}

// Up to 32 antennas: 256 threads, the working matrix in LDS, five workgroups per CU.  Larger
// instances keep the working matrix in the workspace between phases (in registers during the
// sweep), so that LDS holds only the staging buffers: 512 threads and two workgroups per CU up to
// 64 antennas (their latency-bound Gauss-Jordan steps overlap), 1024 threads beyond.
hipError_t launch_setup(const SetupArgs& a, hipStream_t s) {
  if (a.nt <= 32) return launch_setup_bs<256, false, 32>(a, s);
  return a.nt <= 64 ? launch_setup_bs<512, true, 64>(a, s) : launch_setup_bs<1024, true, 128>(a, s);
}

}  // namespace dmala
