// LDS-resident complex FFT and the type-I discrete sine transform built on it.
//
// The lattice Laplacian C^T C of a level is diagonalised by the DST-I of size
// n - 1 along each axis (Sec. 3.2.1 of the paper).  A DST-I of length n - 1 is
// computed here from one complex FFT of length n:
//
//   z  = odd extension of x (length 2n, z_j = x_j, z_{2n-j} = -x_j, z_0 = z_n = 0)
//   w_m = z_{2m} + i z_{2m+1}                      (m = 0 .. n-1)
//   W  = FFT_n(w)
//   E_k = (W_k + conj W_{n-k}) / 2,  O_k = (W_k - conj W_{n-k}) / (2i)
//   X_k = sum_j x_j sin(pi j k / n) = -Im(E_k + e^{-i pi k / n} O_k) / 2
//
// The FFT is a Stockham autosort transform working in place on LDS with stages of the
// largest radix MAXR (16, 8 or 4) first, then one smaller power-of-two stage for the rest
// of the power of two, then radix-3 and radix-5 stages: every stage loads its inputs into registers,
// synchronises the workgroup, and writes the butterflies' outputs back.  Large radices
// mean fewer barriers and less LDS traffic; small ones more butterflies per stage (more
// waves in flight to hide latency) and fewer registers per thread.  The choice is made per
// size by measurement.  Twiddles come from one table per n,
// tw[m] = exp(-i pi m / n), m < 2n, prepared on the host in double precision.
#pragma once

#include "ib_common.hpp"

namespace ib {

constexpr int ilog2c(int m) { return m <= 1 ? 0 : 1 + ilog2c(m / 2); }
constexpr int powc(int l, int f) { return (l % f) ? 0 : 1 + powc(l / f, f); }
constexpr int ipowc(int f, int p) { return p == 0 ? 1 : f * ipowc(f, p - 1); }

template <int L, int MAXR = 16>
struct FftPlan {
  static_assert(MAXR == 16 || MAXR == 8 || MAXR == 4, "largest radix 16, 8 or 4");
  static constexpr int lr = ilog2c(MAXR);
  static constexpr int p5 = powc(L, 5);
  static constexpr int p3 = powc(L / ipowc(5, p5), 3);
  static constexpr int p2 = ilog2c(L / (ipowc(3, p3) * ipowc(5, p5)));
  static constexpr int nbig = p2 / lr;
  static constexpr int rem = p2 % lr;  // one more stage of radix 2^rem
  static constexpr int nmid = rem ? 1 : 0;
  static constexpr int nst = nbig + nmid + p3 + p5;
  static_assert(ipowc(5, p5) * ipowc(3, p3) * (1 << p2) == L, "FFT length must be 2^a 3^b 5^c");
  static constexpr int radix(int s) {
    return s < nbig ? MAXR : (s < nbig + nmid ? (1 << rem) : (s < nbig + nmid + p3 ? 3 : 5));
  }
};

template <typename T>
__device__ __forceinline__ void dft4(c2<T>& a0, c2<T>& a1, c2<T>& a2, c2<T>& a3) {
  c2<T> s02 = cadd(a0, a2), d02 = csub(a0, a2);
  c2<T> s13 = cadd(a1, a3), d13 = csub(a1, a3);
  c2<T> md = cmul_mi(d13);
  a0 = cadd(s02, s13);
  a2 = csub(s02, s13);
  a1 = cadd(d02, md);
  a3 = csub(d02, md);
}

// In-place DFT of R values in natural order, X_k = sum_m v_m e^{-2 pi i m k / R}.
template <typename T, int R>
__device__ __forceinline__ void dft_small(c2<T>* v) {
  if constexpr (R == 2) {
    c2<T> a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  } else if constexpr (R == 4) {
    dft4(v[0], v[1], v[2], v[3]);
  } else if constexpr (R == 8) {
    // even / odd halves, then the twiddles e^{-i pi k / 4}
    c2<T> e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
    c2<T> o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
    dft4(e0, e1, e2, e3);
    dft4(o0, o1, o2, o3);
    const T h = T(0.70710678118654752440084436210485);
    o1 = c2<T>{h * (o1.x + o1.y), h * (o1.y - o1.x)};
    o2 = cmul_mi(o2);
    o3 = c2<T>{h * (o3.y - o3.x), -h * (o3.x + o3.y)};
    v[0] = cadd(e0, o0);
    v[4] = csub(e0, o0);
    v[1] = cadd(e1, o1);
    v[5] = csub(e1, o1);
    v[2] = cadd(e2, o2);
    v[6] = csub(e2, o2);
    v[3] = cadd(e3, o3);
    v[7] = csub(e3, o3);
  } else if constexpr (R == 16) {
    // four DFT4 over m = r + 4 j, the twiddles e^{-2 pi i r k / 16}, four DFT4 over r
#pragma unroll
    for (int r = 0; r < 4; ++r) dft4(v[r], v[r + 4], v[r + 8], v[r + 12]);
    const T c1 = T(0.92387953251128675612818318939679);  // cos(pi/8)
    const T s1 = T(0.38268343236508977172845998403040);  // sin(pi/8)
    const T h = T(0.70710678118654752440084436210485);
    // Y_r[k] sits in v[r + 4k]; multiply by w^{r k}, w = e^{-i pi / 8}
    auto tw = [](c2<T> z, T c, T s) { return c2<T>{z.x * c + z.y * s, z.y * c - z.x * s}; };
    v[5] = tw(v[5], c1, s1);     // r=1 k=1: w^1
    v[9] = tw(v[9], h, h);       // r=1 k=2: w^2
    v[13] = tw(v[13], s1, c1);   // r=1 k=3: w^3
    v[6] = tw(v[6], h, h);       // r=2 k=1: w^2
    v[10] = cmul_mi(v[10]);      // r=2 k=2: w^4
    v[14] = tw(v[14], -h, h);    // r=2 k=3: w^6
    v[7] = tw(v[7], s1, c1);     // r=3 k=1: w^3
    v[11] = tw(v[11], -h, h);    // r=3 k=2: w^6
    v[15] = tw(v[15], -c1, -s1); // r=3 k=3: w^9
#pragma unroll
    for (int k = 0; k < 4; ++k) dft4(v[4 * k], v[4 * k + 1], v[4 * k + 2], v[4 * k + 3]);
    // X[k + 4 q] = DFT4 over r of row k, now in v[4 k + q]: transpose to natural order
    c2<T> u[16];
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
      for (int q = 0; q < 4; ++q) u[k + 4 * q] = v[4 * k + q];
#pragma unroll
    for (int e = 0; e < 16; ++e) v[e] = u[e];
  } else if constexpr (R == 5) {
    // X_k = v_0 + sum_{m=1}^{4} v_m w^{mk}, w = e^{-2 pi i / 5}: pair m with 5 - m, whose
    // twiddles are conjugate (cos(2 pi m k / 5) shared, sin(...) opposite)
    const T c1 = T(0.30901699437494742410229341718282);   // cos(2 pi / 5)
    const T c2v = T(-0.80901699437494742410229341718282); // cos(4 pi / 5)
    const T s1 = T(0.95105651629515357211643933337938);   // sin(2 pi / 5)
    const T s2 = T(0.58778525229247312916870595463907);   // sin(4 pi / 5)
    const c2<T> a1 = cadd(v[1], v[4]), b1 = csub(v[1], v[4]);
    const c2<T> a2 = cadd(v[2], v[3]), b2 = csub(v[2], v[3]);
    const c2<T> x0 = v[0];
    // real parts from the sums, -i times the sine parts from the differences
    const c2<T> r1 = c2<T>{x0.x + c1 * a1.x + c2v * a2.x, x0.y + c1 * a1.y + c2v * a2.y};
    const c2<T> r2 = c2<T>{x0.x + c2v * a1.x + c1 * a2.x, x0.y + c2v * a1.y + c1 * a2.y};
    const c2<T> i1 = c2<T>{s1 * b1.x + s2 * b2.x, s1 * b1.y + s2 * b2.y};   // k = 1
    const c2<T> i2 = c2<T>{s2 * b1.x - s1 * b2.x, s2 * b1.y - s1 * b2.y};   // k = 2
    v[0] = c2<T>{x0.x + a1.x + a2.x, x0.y + a1.y + a2.y};
    v[1] = cadd(r1, cmul_mi(i1));
    v[4] = csub(r1, cmul_mi(i1));
    v[2] = cadd(r2, cmul_mi(i2));
    v[3] = csub(r2, cmul_mi(i2));
  } else {
    // e^{-2 pi i / 3} = -1/2 - i sqrt(3)/2
    const T h3 = T(0.86602540378443864676372317075294);
    c2<T> t1 = cadd(v[1], v[2]), t2 = csub(v[1], v[2]);
    c2<T> m = c2<T>{v[0].x - T(0.5) * t1.x, v[0].y - T(0.5) * t1.y};
    c2<T> r = cmul_mi(t2);
    v[0] = cadd(v[0], t1);
    v[1] = c2<T>{m.x + h3 * r.x, m.y + h3 * r.y};
    v[2] = c2<T>{m.x - h3 * r.x, m.y - h3 * r.y};
  }
}

// LDS layout.  A transform of length L occupies fft_pad_len<L>() slots: element x sits
// at fpad(x) = x + x / 16, which keeps the stride-16 stores of a radix-16 stage off a
// single LDS bank.  The twiddle table in LDS holds first tu[k] = e^{-i pi k / L},
// k = 0 .. L/2 (for the sine-transform unpacking), then, for every stage with NS > 1,
// its (R - 1) NS factors e^{-2 pi i r k / (NS R)} at [(r - 1) NS + k], so that the
// lanes of a wave read consecutive entries.
template <int L>
constexpr int fft_pad_len() { return L + L / 16; }
__device__ __forceinline__ int fpad(int x) { return x + (x >> 4); }

template <int L, int MAXR = 16>
struct TwLayout {
  static constexpr int U = L / 2 + 1;
  static constexpr int off(int S) {
    int o = U, ns = 1;
    for (int s = 0; s < S; ++s) {
      const int r = FftPlan<L, MAXR>::radix(s);
      if (ns > 1) o += (r - 1) * ns;
      ns *= r;
    }
    return o;
  }
  static constexpr int total = off(FftPlan<L, MAXR>::nst);
};

// Index into the global table exp(-i pi m / L), m < 2L, of LDS table entry e.
template <int L, int MAXR = 16, int S = 0, int NS = 1>
__device__ __forceinline__ int tw_source(int e) {
  if constexpr (S >= FftPlan<L, MAXR>::nst) {
    return 0;
  } else {
    constexpr int R = FftPlan<L, MAXR>::radix(S);
    constexpr int O = TwLayout<L, MAXR>::off(S);
    if (NS > 1 && e >= O && e < O + (R - 1) * NS) {
      const int q = e - O, r = 1 + q / NS, k = q % NS;
      return ((2 * L) / (NS * R)) * r * k;
    }
    return tw_source<L, MAXR, S + 1, NS * R>(e);
  }
}

// One Stockham stage S on COUNT transforms of length L stored back to back in buf.
template <typename T, int L, int MAXR, int S, int R, int NS, int COUNT, int NT>
__device__ __forceinline__ void fft_stage(c2<T>* buf, const c2<T>* __restrict__ tws, int tid) {
  constexpr int LR = L / R;
  constexpr int NB = COUNT * LR;
  constexpr int PER = (NB + NT - 1) / NT;
  constexpr int PL = fft_pad_len<L>();
  constexpr int TO = TwLayout<L, MAXR>::off(S);
  c2<T> v[PER][R];
#pragma unroll
  for (int b = 0; b < PER; ++b) {
    int jj = tid + b * NT;
    if (jj < NB) {
      int t = jj / LR, j = jj % LR;
      const c2<T>* base = buf + t * PL;
#pragma unroll
      for (int r = 0; r < R; ++r) v[b][r] = base[fpad(j + r * LR)];
    }
  }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < PER; ++b) {
    int jj = tid + b * NT;
    if (jj < NB) {
      int t = jj / LR, j = jj % LR;
      int k = j % NS;
      if constexpr (NS > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) v[b][r] = cmul(v[b][r], tws[TO + (r - 1) * NS + k]);
      }
      dft_small<T, R>(v[b]);
      int d = (j / NS) * NS * R + k;
      c2<T>* base = buf + t * PL;
#pragma unroll
      for (int r = 0; r < R; ++r) base[fpad(d + r * NS)] = v[b][r];
    }
  }
  __syncthreads();
}

template <typename T, int L, int MAXR, int S, int NS, int COUNT, int NT>
__device__ __forceinline__ void fft_run(c2<T>* buf, const c2<T>* __restrict__ tws, int tid) {
  if constexpr (S < FftPlan<L, MAXR>::nst) {
    constexpr int R = FftPlan<L, MAXR>::radix(S);
    fft_stage<T, L, MAXR, S, R, NS, COUNT, NT>(buf, tws, tid);
    fft_run<T, L, MAXR, S + 1, NS * R, COUNT, NT>(buf, tws, tid);
  }
}

// Forward complex FFT (e^{-2 pi i m k / L}) of COUNT sequences in LDS (padded layout,
// natural order); tws is the LDS table described above.  Requires a workgroup barrier
// before (inputs written) and leaves one after.
template <typename T, int L, int COUNT, int NT, int MAXR = 16>
__device__ __forceinline__ void fft_lds(c2<T>* buf, const c2<T>* __restrict__ tws, int tid) {
  fft_run<T, L, MAXR, 0, 1, COUNT, NT>(buf, tws, tid);
}

// Place x_j (j = 1 .. n-1) of one sequence into its packed odd extension w.
template <typename T, int N>
__device__ __forceinline__ void dst_pack(c2<T>* w, int j, T xj) {
  T* wr = reinterpret_cast<T*>(w);
  // z_j lives in w[j/2] (real part if j even), z_{2n-j} = -x_j in w[(2n-j)/2]
  wr[2 * fpad(j >> 1) + (j & 1)] = xj;
  int jm = 2 * N - j;
  wr[2 * fpad(jm >> 1) + (jm & 1)] = -xj;
}

// Zero the two packed slots that hold z_0 and z_n.
template <typename T, int N>
__device__ __forceinline__ void dst_pack_zeros(c2<T>* w) {
  T* wr = reinterpret_cast<T*>(w);
  wr[0] = T(0);
  wr[2 * fpad(N >> 1)] = T(0);
}

// Unpack the DST-I outputs X_k and X_{n-k} (k = 1 .. n/2) from W = FFT_n(w).
// Returns them through xk, xnk (for k = n/2 both hold X_{n/2}).  tws: LDS table.
template <typename T, int N>
__device__ __forceinline__ void dst_unpack(const c2<T>* W, const c2<T>* __restrict__ tws, int k,
                                           T& xk, T& xnk) {
  c2<T> a = W[fpad(k)];
  c2<T> b = W[fpad(N - k)];
  // E = (a + conj b)/2, O = -i (a - conj b) / 2
  T e_im = T(0.5) * (a.y - b.y);
  c2<T> d = c2<T>{a.x - b.x, a.y + b.y};
  c2<T> o = c2<T>{T(0.5) * d.y, -T(0.5) * d.x};
  c2<T> p = cmul(tws[k], o);
  xk = -T(0.5) * (e_im + p.y);
  xnk = T(0.5) * (e_im - p.y);
}

// sin(pi k / n) for 0 <= k <= n from the LDS table (the table holds k <= n/2).
template <typename T, int N>
__device__ __forceinline__ T tw_sin(const c2<T>* __restrict__ tws, int k) {
  return -tws[k <= N / 2 ? k : N - k].y;
}

}  // namespace ib
