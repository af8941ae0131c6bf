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
#include <type_traits>

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
typedef double d4 __attribute__((ext_vector_type(4)));
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

constexpr int kRedSlots = 16;   // one per wavefront of a workgroup of up to 1024 threads

// Sum (or maximum) of v over the workgroup, returned to every thread: a butterfly within each
// wavefront, then one pass over the per-wave partials in a fixed order (two barriers).
__device__ double block_reduce(double v, double* red, bool is_max) {
  const int tid = threadIdx.x, nw = (blockDim.x + 63) >> 6;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const double u = __shfl_xor(v, o, 64);
    v = is_max ? fmax(v, u) : v + u;
  }
  if ((tid & 63) == 0) red[tid >> 6] = v;
  __syncthreads();
  double r = red[0];
  for (int w = 1; w < nw; ++w) r = is_max ? fmax(r, red[w]) : r + red[w];
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
// The form (NPASS terms, bf16, complex planes) is a compile-time choice and the function is inlined,
// so that the element loop has no branches and X keeps its address space (LDS reads, not flat loads).
template <int NPASS, bool BF16, bool CX>
__device__ __forceinline__ float pack_fragments(const cd* X, int ld, double c, int nt, int N, int RT, int KB,
                                                unsigned char* dst) {
  constexpr int npass = NPASS;
  constexpr bool bf16 = BF16, cx = CX;
  // X is Hermitian positive semidefinite (G, and A = I - gamma M, whose eigenvalues lie in [0, 1)),
  // so |Re x_ij|, |Im x_ij| <= |x_ij| <= sqrt(x_ii x_jj) <= max_i x_ii: the largest entry is the
  // largest diagonal one.  Every wavefront reads the diagonal and reduces it for itself (no barrier).
  double mx = 0.0;
  for (int i = threadIdx.x & 63; i < nt; i += 64) mx = fmax(mx, fabs(X[i * ld + i].re));
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
  mx *= fabs(c);
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
      if constexpr (cx) {
        const cd e = X[(n < nt && n2 < nt ? n : 0) * ld + (n2 < nt ? n2 : 0)];
        v = (n < nt && n2 < nt) ? sc * (pl ? e.im : e.re) : 0.0;
      } else {
        v = (n < N && n2 < N) ? sc * realeq(X, ld, n, n2) : 0.0;
      }
      if constexpr (bf16) {
        f0.b[j] = (__bf16)via_float(v);
      } else {
        const _Float16 hi = (_Float16)via_float(v);
        const double r1 = v - (double)hi;
        const _Float16 mid = (_Float16)via_float(r1);
        const double r2 = r1 - (double)mid;
        if constexpr (npass == 3) { f0.h[j] = (_Float16)via_float(r2); f1.h[j] = mid; f2.h[j] = hi; }
        else if constexpr (npass == 2) { f0.h[j] = mid; f1.h[j] = hi; }
        else f0.h[j] = hi;
      }
    }
    unsigned char* o = dst + (size_t)t * 1024 + l * 16;
    *(uint4*)o = f0.u;
    if constexpr (npass > 1) *(uint4*)(o + pass_stride) = f1.u;
    if constexpr (npass > 2) *(uint4*)(o + 2 * pass_stride) = f2.u;
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

// Working-matrix placement and thread counts (launch_setup): up to 64 antennas 256 threads with the
// matrix in LDS (up to about 75 KiB: two workgroups per CU), beyond that 1024 threads with the
// matrix in this instance's slice of the workspace.
// RMAX: rows of the working matrix the Gauss-Jordan register layout covers (threads per row BS / RMAX).
template <typename TIn, bool WGLOB, int BS, int RMAX>
__device__ __forceinline__ void setup_body(const SetupArgs& a, const int b) {
  const int tid = threadIdx.x, nt = a.nt, nr = a.nr, N = a.N, Npad = a.Npad;
  const int ld = nt + 1;  // padded leading dimension of the matrices (no LDS bank conflicts on columns)
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
  cd* rowp = bv + nt;       // 2 x 2 x nt (alternating Gauss-Jordan steps, two pivot rows each)
  cd* colp = rowp + 4 * nt; // 2 x 2 x nt
  double* red = (double*)(colp + 4 * nt);   // kRedSlots partials of block_reduce
  unsigned char* blk = a.ws_inst + (size_t)b * a.inst_stride;

  const int Q = a.Q, M = Q * Q;
  const double s = sqrt(3.0 / (2.0 * (M - 1)));
  const double tau = a.tau;
  const double alpha = a.alpha_mult * sigma2;
  const double beta = a.naive ? 1.0 : a.beta_mult * s * s / sigma2;
  const double gamma = a.gamma_mult * sigma2 / (2.0 * s * s);

  // G = H^H H and z = H^H y.  H is staged in LDS in chunks of receive antennas,
  // transposed with a padded row whose last entry holds y (Ht[i][m], Ht[i][nt] = y_i).
  // G on the matrix cores: with X = Re + i Im of the staged H^T (nt x nr),
  //   Re G = Re Re^T + Im Im^T,   Im G = Re Im^T - Im Re^T,
  // four float64 16x16x4 MFMAs per 16 x 16 tile and 4 receive antennas; each wave
  // accumulates the upper-triangle tiles (tr <= tc) assigned to it in registers across
  // the chunks and writes the tile and its conjugate transpose.  z on the vector ALUs:
  // P = BS / RMAX consecutive threads share an antenna m and split the receive
  // antennas, then sum over those lanes.
  double nonfinite = 0.0;
  double yy = 0.0;
  {
    constexpr int kIC = RMAX <= 32 ? 16 : 32;
    constexpr int NW = BS / 64;
    constexpr int kNT = (RMAX + 15) / 16;                         // tile rows at nt = RMAX
    constexpr int kTPW = (kNT * (kNT + 1) / 2 + NW - 1) / NW;     // tiles per wave
    constexpr int P = BS / RMAX;
    static_assert(P >= 1 && 64 % P == 0, "the threads of an antenna share a wavefront");
    // kIC x ld, then one spare row; with the working matrix in LDS (33 to 64
    // antennas) the staging buffer is its first rows, written only after the last read
    cd* Ht = (!WGLOB && RMAX > 32) ? W : (cd*)(red + kRedSlots);
    const int lane = tid & 63, wv = tid >> 6;
    const int ntr = (nt + 15) >> 4, ntiles = ntr * (ntr + 1) / 2;
    int m0[kTPW], m1[kTPW];
    d4 gre[kTPW], gim[kTPW];
#pragma unroll
    for (int q = 0; q < kTPW; ++q) {
      int t = wv + q * NW, tr = 0;
      if (t >= ntiles) t = 0;
      while (t >= ntr - tr) { t -= ntr - tr; ++tr; }
      m0[q] = 16 * tr;
      m1[q] = 16 * (tr + t);
      gre[q] = d4{0.0, 0.0, 0.0, 0.0};
      gim[q] = d4{0.0, 0.0, 0.0, 0.0};
    }
    const int zm = tid / P, zp = tid % P;
    cd zacc = {0.0, 0.0};
    // The chunk of receive antennas i0 .. i0 + kIC - 1 is loaded into registers (every load
    // issued before the first is waited for), then stored to LDS; the next chunk's loads are
    // issued before this chunk's products, so that they overlap.  Element e of a chunk:
    // receive antenna i0 + e % kIC, column e / kIC (column nt: y).
    constexpr int kSt = (kIC * (RMAX + 1) + BS - 1) / BS;
    TIn hv[kSt][2];
    auto load_chunk = [&](int i0) {
      const int ic = nr - i0 < kIC ? nr - i0 : kIC;
#pragma unroll
      for (int k = 0; k < kSt; ++k) {
        const int e = tid + k * BS, mm = e / kIC, ii = e % kIC;
        if (mm <= nt && ii < ic) {
          const TIn* src = mm < nt ? Hg + 2 * ((size_t)mm * nr + i0 + ii) : y + 2 * (i0 + ii);
          hv[k][0] = src[0];
          hv[k][1] = src[1];
        }
      }
    };
    load_chunk(0);
    for (int i0 = 0; i0 < nr; i0 += kIC) {
      const int ic = nr - i0 < kIC ? nr - i0 : kIC;
#pragma unroll
      for (int k = 0; k < kSt; ++k) {
        const int e = tid + k * BS, mm = e / kIC, ii = e % kIC;
        if (mm <= nt && ii < ic) Ht[ii * ld + mm] = {(double)hv[k][0], (double)hv[k][1]};
      }
      __syncthreads();
      if (i0 + kIC < nr) load_chunk(i0 + kIC);
      // |y|^2 from the staged y
      if (tid < ic) {
        const cd yv = Ht[tid * ld + nt];
        yy = fma(yv.re, yv.re, fma(yv.im, yv.im, yy));
      }
#pragma unroll
      for (int q = 0; q < kTPW; ++q) {
        if (wv + q * NW < ntiles) {
          const int ra = m0[q] + (lane & 15), rb = m1[q] + (lane & 15);
          for (int kk = 0; kk < ic; kk += 4) {
            const int ii = kk + (lane >> 4);
            const bool ok = ii < ic;
            const cd va = (ok && ra < nt) ? Ht[ii * ld + ra] : cd{0.0, 0.0};
            const cd vb = (ok && rb < nt) ? Ht[ii * ld + rb] : cd{0.0, 0.0};
            gre[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(va.re, vb.re, gre[q], 0, 0, 0);
            gre[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(va.im, vb.im, gre[q], 0, 0, 0);
            gim[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(va.re, vb.im, gim[q], 0, 0, 0);
            gim[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(-va.im, vb.re, gim[q], 0, 0, 0);
          }
        }
      }
      if (zm < nt) {
        for (int ii = zp; ii < ic; ii += P) {
          const cd h = Ht[ii * ld + zm], yv = Ht[ii * ld + nt];
          zacc.re = fma(h.re, yv.re, fma(h.im, yv.im, zacc.re));
          zacc.im = fma(h.re, yv.im, fma(-h.im, yv.re, zacc.im));
        }
      }
      __syncthreads();
    }
#pragma unroll
    for (int o = P >> 1; o > 0; o >>= 1) {
      zacc.re += __shfl_xor(zacc.re, o, 64);
      zacc.im += __shfl_xor(zacc.im, o, 64);
    }
    if (zm < nt && zp == 0) {
      z[zm] = zacc;
      if (!isfinite(zacc.re) || !isfinite(zacc.im)) nonfinite = 1.0;
    }
    // lane l, register j of a tile's accumulator: row l / 16 + 4 j, column l % 16
#pragma unroll
    for (int q = 0; q < kTPW; ++q) {
      if (wv + q * NW < ntiles) {
        const int col = m1[q] + (lane & 15);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int row = m0[q] + (lane >> 4) + 4 * j;
          if (row < nt && col < nt) {
            const double re = gre[q][j], im = gim[q][j];
            W[row * ld + col] = {re, im};
            if (m0[q] != m1[q]) W[col * ld + row] = {re, -im};
            if (!isfinite(re) || !isfinite(im)) nonfinite = 1.0;
          }
        }
      }
    }
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
    unsigned char* fe = frag + (size_t)npP * pass_bytes;
    scaleE = a.cx ? pack_fragments<kEPasses, false, true>(W, ld, cE, nt, N, a.RT, a.KB, fe)
                  : pack_fragments<kEPasses, false, false>(W, ld, cE, nt, N, a.RT, a.KB, fe);
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
    // W <- (G + gamma I)^-1 by in-place Gauss-Jordan with the working matrix in
    // registers, in SR x SC blocks on a TR x TC thread grid: thread (ti, tj) keeps
    // rows ti + TR a (a < SR) and columns tj + TC c (c < SC) for the whole sweep.  A
    // step on pivot p: the owners of column p publish it (colp); the threads of row
    // p, which share a wavefront with the pivot, read the pivot from its lane, scale
    // their row by its inverse (the inverse itself in column p) and publish it
    // (rowp); after one barrier every other row i clears its column p and subtracts
    // colp[i] * rowp, which leaves -w_ip / w_pp there.  Per step a thread reads SC
    // entries of the row vector and SR of the column for SR SC updates.  The steps on
    // different pivots commute (G + gamma I is Hermitian positive definite, so every
    // pivot stays nonzero in any order), so they run in the order p = o + TR kb, o
    // outer: row p then sits in register slot kb and column p in slot kb / (TC / TR)
    // of thread column o + TR (kb % (TC / TR)), compile-time indices of the unrolled
    // inner loop.  The two vectors alternate between steps, so one barrier per step
    // orders all reads and writes.
    constexpr int TR = BS >= 1024 ? 32 : 16;
    constexpr int TC = BS / TR;
    constexpr int SR = RMAX / TR, SC = RMAX / TC;
    static_assert(TR * TC == BS && SR * TR == RMAX && SC * TC == RMAX && TC % TR == 0 && 64 % TC == 0,
                  "thread grid: a row's threads in one wavefront");
    const int ti = tid / TC, tj = tid % TC;
    cd w[SR][SC];
#pragma unroll
    for (int ra = 0; ra < SR; ++ra)
#pragma unroll
      for (int c = 0; c < SC; ++c) {
        const int i = ti + TR * ra, j = tj + TC * c;
        w[ra][c] = (i < nt && j < nt) ? W[i * ld + j] : cd{0.0, 0.0};
        if (i == j && i < nt) w[ra][c].re += gamma;
      }
    // Pivots are taken two at a time where they can be (rows p and p + 1 of the same
    // register slot, owned by thread rows o and o + 1 of one wavefront): the 2 x 2
    // pivot block B is inverted in registers, rows p and p + 1 become B^-1 times
    // themselves (the partner row's entries come from lane + TC), and every other row
    // subtracts colp0[i] * rowp0 + colp1[i] * rowp1 -- one barrier per two pivots.
    // (1024 threads: single pivots, as the pair step would not fit in 128 registers.)
    constexpr bool kPair = BS < 1024;
    int par = 0;
#pragma unroll 1
    for (int o = 0; o < TR && o < nt; o += kPair ? 2 : 1) {
#pragma unroll
      for (int kb = 0; kb < SR; ++kb) {
        const int p = o + TR * kb;
        if (p >= nt) continue;
        constexpr int kR = TC / TR;
        const int cs = kb / kR;              // column slot of p (compile time)
        const int po = o + TR * (kb % kR);   // thread column that owns column p
        cd* rp = rowp + par * 2 * nt;
        cd* cp = colp + par * 2 * nt;
        par ^= 1;
        if (kPair && p + 1 < nt) {
          if (tj == po || tj == po + 1) {
            cd* cpx = cp + (tj == po ? 0 : nt);
#pragma unroll
            for (int ra = 0; ra < SR; ++ra)
              if (ti + TR * ra < nt) cpx[ti + TR * ra] = w[ra][cs];
          }
          if (tid >> 6 == (o * TC) >> 6) {   // the wavefront of rows p and p + 1
            const int l0 = (o * TC + po) & 63;
            const cd pa = {readlane_f64(w[kb][cs].re, l0), readlane_f64(w[kb][cs].im, l0)};
            const cd pb = {readlane_f64(w[kb][cs].re, l0 + 1), readlane_f64(w[kb][cs].im, l0 + 1)};
            const cd pc = {readlane_f64(w[kb][cs].re, l0 + TC), readlane_f64(w[kb][cs].im, l0 + TC)};
            const cd pd = {readlane_f64(w[kb][cs].re, l0 + TC + 1), readlane_f64(w[kb][cs].im, l0 + TC + 1)};
            const cd det = {pa.re * pd.re - pa.im * pd.im - (pb.re * pc.re - pb.im * pc.im),
                            pa.re * pd.im + pa.im * pd.re - (pb.re * pc.im + pb.im * pc.re)};
            const double rd = 1.0 / (det.re * det.re + det.im * det.im);
            const cd idet = {det.re * rd, -det.im * rd};
            const cd q00 = cmul(pd, idet), q11 = cmul(pa, idet);
            const cd q01 = cmul({-pb.re, -pb.im}, idet), q10 = cmul({-pc.re, -pc.im}, idet);
            const bool top = ti == o;
            const cd qs = top ? q00 : q11, qo = top ? q01 : q10;   // own row, partner row
#pragma unroll
            for (int c = 0; c < SC; ++c) {
              const cd oth = {__shfl_xor(w[kb][c].re, TC, 64), __shfl_xor(w[kb][c].im, TC, 64)};
              if (ti == o || ti == o + 1) w[kb][c] = cadd(cmul(qs, w[kb][c]), cmul(qo, oth));
            }
            if (ti == o || ti == o + 1) {
              if (tj == po) w[kb][cs] = top ? q00 : q10;
              if (tj == po + 1) w[kb][cs] = top ? q01 : q11;
              cd* rpx = rp + (top ? 0 : nt);
#pragma unroll
              for (int c = 0; c < SC; ++c)
                if (tj + TC * c < nt) rpx[tj + TC * c] = w[kb][c];
            }
          }
          __syncthreads();
          // row entries past column nt - 1 read whatever follows the row vectors in LDS
          // (inside the allocation); they update register entries that are never stored
          cd r0[SC], r1[SC];
#pragma unroll
          for (int c = 0; c < SC; ++c) {
            r0[c] = rp[tj + TC * c];
            r1[c] = rp[nt + tj + TC * c];
          }
#pragma unroll
          for (int ra = 0; ra < SR; ++ra) {
            const int i = ti + TR * ra;
            if (i < nt && i != p && i != p + 1) {
              const cd c0 = cp[i], c1 = cp[nt + i];
              if (tj == po || tj == po + 1) w[ra][cs] = {0.0, 0.0};
#pragma unroll
              for (int c = 0; c < SC; ++c) {
                cd& v = w[ra][c];
                v.re = fma(-c0.re, r0[c].re, fma(c0.im, r0[c].im, v.re));
                v.im = fma(-c0.re, r0[c].im, fma(-c0.im, r0[c].re, v.im));
                v.re = fma(-c1.re, r1[c].re, fma(c1.im, r1[c].im, v.re));
                v.im = fma(-c1.re, r1[c].im, fma(-c1.im, r1[c].re, v.im));
              }
            }
          }
        } else {
          // a single pivot (1024 threads, or the last row of a slot that nt leaves unpaired)
          if (tj == po) {
#pragma unroll
            for (int ra = 0; ra < SR; ++ra)
              if (ti + TR * ra < nt) cp[ti + TR * ra] = w[ra][cs];
          }
          if (ti == o) {
            const int l0 = (o * TC + po) & 63;
            const cd piv = {readlane_f64(w[kb][cs].re, l0), readlane_f64(w[kb][cs].im, l0)};
            const double rd = 1.0 / (piv.re * piv.re + piv.im * piv.im);
            const cd inv = {piv.re * rd, -piv.im * rd};
#pragma unroll
            for (int c = 0; c < SC; ++c) w[kb][c] = cmul(w[kb][c], inv);
            if (tj == po) w[kb][cs] = inv;
#pragma unroll
            for (int c = 0; c < SC; ++c)
              if (tj + TC * c < nt) rp[tj + TC * c] = w[kb][c];
          }
          __syncthreads();
          cd r[SC];
#pragma unroll
          for (int c = 0; c < SC; ++c) r[c] = rp[tj + TC * c];
#pragma unroll
          for (int ra = 0; ra < SR; ++ra) {
            const int i = ti + TR * ra;
            if (i < nt && i != p) {
              const cd ci = cp[i];
              if (tj == po) w[ra][cs] = {0.0, 0.0};
#pragma unroll
              for (int c = 0; c < SC; ++c) {
                cd& v = w[ra][c];
                v.re = fma(-ci.re, r[c].re, fma(ci.im, r[c].im, v.re));
                v.im = fma(-ci.re, r[c].im, fma(-ci.im, r[c].re, v.im));
              }
            }
          }
        }
      }
    }
    // From the registers of M's blocks: b = M z (each thread's columns, then summed over the TC
    // threads of a row, which every one of them ends with bit for bit), the preconditioned
    // variance feature from M's diagonal, and A = I - gamma M written back over the matrix.
    float* afv = (float*)(frag + (size_t)(npP + kEPasses) * pass_bytes) + 2 * Npad;
    cd zc[SC];
#pragma unroll
    for (int c = 0; c < SC; ++c) zc[c] = tj + TC * c < nt ? z[tj + TC * c] : cd{0.0, 0.0};
#pragma unroll
    for (int ra = 0; ra < SR; ++ra) {
      const int i = ti + TR * ra;
      cd bp = {0.0, 0.0};
#pragma unroll
      for (int c = 0; c < SC; ++c) {
        const int j = tj + TC * c;
        // register entries of columns j >= nt hold whatever the sweep read past the row
        // vectors (possibly not finite): they are left out, not multiplied by zero
        if (j < nt) bp = cadd(bp, cmul(w[ra][c], zc[c]));
        if (i < nt && j < nt) W[i * ld + j] = {(j == i ? 1.0 : 0.0) - gamma * w[ra][c].re, -gamma * w[ra][c].im};
      }
#pragma unroll
      for (int o = TC >> 1; o > 0; o >>= 1) {
        bp.re += __shfl_xor(bp.re, o, 64);
        bp.im += __shfl_xor(bp.im, o, 64);
      }
      if (i < nt && tj == 0) bv[i] = bp;
      // diagonal entry (i, i): thread column ti + TR (ra % (TC / TR)), slot ra / (TC / TR)
      if (i < nt && tj == ti + TR * (ra % (TC / TR)) && !a.fp64)
        afv[2 * i] = (float)(log2(sigma2 * w[ra][ra / (TC / TR)].re / (8.0 * s * s)) / 8.0);
    }
    __syncthreads();
    if (a.fp64) {
      pack_dense(W, ld, cP, N, Npad, (double*)(blk + kParamBytes));
      double* pbd = (double*)(blk + kParamBytes) + 2 * (size_t)Npad * Npad;
      for (int n = tid; n < Npad; n += blockDim.x) pbd[n] = n < N ? cb * realeq_vec(bv, n) : 0.0;
    } else {
      auto packP = [&](auto CXC) {
        constexpr bool C = decltype(CXC)::value;
        if (a.pm == PM_BF16X1) return pack_fragments<1, true, C>(W, ld, cP, nt, N, a.RT, a.KB, frag);
        if (npP == 2) return pack_fragments<2, false, C>(W, ld, cP, nt, N, a.RT, a.KB, frag);
        return pack_fragments<1, false, C>(W, ld, cP, nt, N, a.RT, a.KB, frag);
      };
      scaleP = a.cx ? packP(std::true_type{}) : packP(std::false_type{});
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

// Direct launch (PERS false): instance blockIdx.x.  Persistent launch: items from the list, each
// with its class's arguments.
template <typename TIn, bool WGLOB, int BS, int RMAX, bool PERS = false>
__global__ __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(RMAX <= 32 ? 5 : (BS == 512 ? 4 : (BS == 256 ? 2 : 1)))))
void setup_kernel(SetupArgs a, Persist p) {
  if constexpr (!PERS) {
    setup_body<TIn, WGLOB, BS, RMAX>(a, blockIdx.x);
  } else {
    extern __shared__ double smem_setup[];
    for (;;) {
      const int it = persist_take(p, (unsigned char*)smem_setup);
      if (it >= p.n_items) break;
      const WorkItem w = p.items[it];
      const SetupArgs ca = ((const SetupArgs*)p.cls)[__builtin_amdgcn_readfirstlane(w.cls)];
      setup_body<TIn, WGLOB, BS, RMAX>(ca, __builtin_amdgcn_readfirstlane(w.inst));
    }
    persist_done(p);
  }
}

bool setup_w_global(int nt) { return nt > 64; }

template <int BS, bool WG, int RMAX>
hipError_t launch_setup_bs(const SetupArgs& a, hipStream_t s, const Persist* p, int gn, KernelCfg* cfg) {
  if (WG != setup_w_global(a.nt) || a.nt > RMAX) return hipErrorInvalidValue;
  constexpr int kIC = RMAX <= 32 ? 16 : 32;
  const bool alias = !WG && RMAX > 32;   // the staging buffer is the working matrix's first rows
  const size_t lds = (size_t)((WG ? 0 : a.nt * (a.nt + 1)) + 10 * a.nt) * sizeof(cd) + kRedSlots * sizeof(double) +
                     (alias ? 0 : (kIC * (size_t)(a.nt + 1) + 32) * sizeof(cd));
  void (*k)(SetupArgs, Persist);
  if (p || cfg) k = a.fp64 ? setup_kernel<double, WG, BS, RMAX, true> : setup_kernel<float, WG, BS, RMAX, true>;
  else k = a.fp64 ? setup_kernel<double, WG, BS, RMAX> : setup_kernel<float, WG, BS, RMAX>;
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

// Up to 32 antennas: 256 threads, the working matrix in LDS, five workgroups per CU.  Up to 64
// antennas: 256 threads, the working matrix in LDS (about 75 KiB with the other vectors), two
// workgroups per CU whose latency-bound Gauss-Jordan steps overlap.  Larger instances keep the
// working matrix in the workspace between phases (in registers during the sweep), so that LDS
// holds only the staging buffers: 1024 threads.
hipError_t launch_setup(const SetupArgs& a, hipStream_t s, const Persist* p, int gn, KernelCfg* cfg) {
  if (a.nt <= 32) return launch_setup_bs<256, false, 32>(a, s, p, gn, cfg);
  return a.nt <= 64 ? launch_setup_bs<512, false, 64>(a, s, p, gn, cfg) : launch_setup_bs<1024, true, 128>(a, s, p, gn, cfg);
}

}  // namespace dmala
