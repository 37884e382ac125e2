// zk_fft.hpp -- Stockham FFT for one team of T threads (T a power of two, 32 to 1024).
//
// A team transforms one sequence of N = E * T complex points.  Thread t holds
// the E elements t + T*r in registers on entry; the first pass is a radix-E
// butterfly entirely in registers (E = 3, 6 or 12 for the 3/2-padded lengths
// 3*2^k, E = 2, 4 or 8 for the base lengths 2^k); the remaining radix-4/2
// passes exchange through LDS (Stockham autosort: natural order in, natural
// order out).  team_fft leaves the result in LDS for the caller to read in
// whatever element-to-thread mapping it needs; team_fft_keep leaves it in
// registers in the last pass's layout, and team_fft_t (the transposed
// algorithm) takes its input in that layout and returns the result in the
// t + T*r layout, each one LDS round trip fewer.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

namespace zk {

template <typename R>
struct cpx {
  R x, y;
};

template <typename R>
__device__ __forceinline__ cpx<R> cadd(cpx<R> a, cpx<R> b) { return {a.x + b.x, a.y + b.y}; }
template <typename R>
__device__ __forceinline__ cpx<R> csub(cpx<R> a, cpx<R> b) { return {a.x - b.x, a.y - b.y}; }
template <typename R>
__device__ __forceinline__ cpx<R> cmul(cpx<R> a, cpx<R> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename R>
__device__ __forceinline__ cpx<R> cscale(cpx<R> a, R s) { return {a.x * s, a.y * s}; }
template <typename R>
__device__ __forceinline__ cpx<R> cconj(cpx<R> a) { return {a.x, -a.y}; }
// multiply by (DIR * i)
template <int DIR, typename R>
__device__ __forceinline__ cpx<R> mul_diri(cpx<R> a) {
  if constexpr (DIR > 0) return {-a.y, a.x};
  else return {a.y, -a.x};
}

// cos and sin of 2 pi j / 48 (quarter turns are special-cased exactly)
__host__ __device__ constexpr double cos48(int j) {
  constexpr double tab[48] = {
    1, 0.99144486137381038, 0.96592582628906831, 0.92387953251128674,
    0.8660254037844386, 0.79335334029123517, 0.70710678118654757, 0.60876142900872066,
    0.5, 0.38268343236508978, 0.25881904510252074, 0.1305261922200516,
    0, -0.1305261922200516, -0.25881904510252074, -0.38268343236508978,
    -0.5, -0.60876142900872066, -0.70710678118654757, -0.79335334029123517,
    -0.8660254037844386, -0.92387953251128674, -0.96592582628906831, -0.99144486137381038,
    -1, -0.99144486137381038, -0.96592582628906831, -0.92387953251128674,
    -0.8660254037844386, -0.79335334029123517, -0.70710678118654757, -0.60876142900872066,
    -0.5, -0.38268343236508978, -0.25881904510252074, -0.1305261922200516,
    0, 0.1305261922200516, 0.25881904510252074, 0.38268343236508978,
    0.5, 0.60876142900872066, 0.70710678118654757, 0.79335334029123517,
    0.8660254037844386, 0.92387953251128674, 0.96592582628906831, 0.99144486137381038};
  return tab[j];
}
__host__ __device__ constexpr double sin48(int j) {
  constexpr double tab[48] = {
    0, 0.1305261922200516, 0.25881904510252074, 0.38268343236508978,
    0.5, 0.60876142900872066, 0.70710678118654757, 0.79335334029123517,
    0.8660254037844386, 0.92387953251128674, 0.96592582628906831, 0.99144486137381038,
    1, 0.99144486137381038, 0.96592582628906831, 0.92387953251128674,
    0.8660254037844386, 0.79335334029123517, 0.70710678118654757, 0.60876142900872066,
    0.5, 0.38268343236508978, 0.25881904510252074, 0.1305261922200516,
    0, -0.1305261922200516, -0.25881904510252074, -0.38268343236508978,
    -0.5, -0.60876142900872066, -0.70710678118654757, -0.79335334029123517,
    -0.8660254037844386, -0.92387953251128674, -0.96592582628906831, -0.99144486137381038,
    -1, -0.99144486137381038, -0.96592582628906831, -0.92387953251128674,
    -0.8660254037844386, -0.79335334029123517, -0.70710678118654757, -0.60876142900872066,
    -0.5, -0.38268343236508978, -0.25881904510252074, -0.1305261922200516};
  return tab[j];
}

// cos and sin of 2 pi m / n for any compile-time m, n: the angle is reduced
// exactly in integers to [0, pi/4] (octant symmetries), then a Taylor series
// in long double, far below double rounding at |x| <= pi/4.
constexpr long double kPiL = 3.14159265358979323846264338327950288L;
constexpr long double taylor_cos(long double x) {
  long double t = 1.0L, s = 1.0L;
  for (int k = 1; k < 12; ++k) {
    t *= -x * x / ((2 * k - 1) * (2 * k));
    s += t;
  }
  return s;
}
constexpr long double taylor_sin(long double x) {
  long double t = x, s = x;
  for (int k = 1; k < 12; ++k) {
    t *= -x * x / ((2 * k) * (2 * k + 1));
    s += t;
  }
  return s;
}
// (cos, sin) of 2 pi m / n, 0 <= m < n: with 8m = o n + r (octant o, 0 <= r < n),
// the angle is o pi/4 + (pi/4) r / n.
constexpr double cos_sin_frac(int m, int n, bool want_sin) {
  const long long a = 8LL * m;
  const int o = (int)(a / n);
  const long double x = kPiL / 4 * (long double)(a % n) / n;  // in [0, pi/4)
  const long double c = taylor_cos(x), sn = taylor_sin(x);
  const long double h = 0.70710678118654752440084436210484903928L;  // cos(pi/4)
  long double cc = 0, ss = 0;
  switch (o) {  // rotate (c, sn) by o pi/4
    case 0: cc = c; ss = sn; break;
    case 1: cc = h * (c - sn); ss = h * (c + sn); break;
    case 2: cc = -sn; ss = c; break;
    case 3: cc = -h * (c + sn); ss = h * (c - sn); break;
    case 4: cc = -c; ss = -sn; break;
    case 5: cc = -h * (c - sn); ss = -h * (c + sn); break;
    case 6: cc = sn; ss = -c; break;
    default: cc = h * (c + sn); ss = -h * (c - sn); break;
  }
  return (double)(want_sin ? ss : cc);
}

// a * exp(DIR * 2 pi i * M / NN) for compile-time M, NN
template <int M, int NN, int DIR, typename R>
__device__ __forceinline__ cpx<R> twc(cpx<R> a) {
  constexpr int mm = ((M % NN) + NN) % NN;
  if constexpr (mm == 0) {
    return a;
  } else if constexpr (4 * mm == NN) {
    return mul_diri<DIR>(a);
  } else if constexpr (2 * mm == NN) {
    return {-a.x, -a.y};
  } else if constexpr (4 * mm == 3 * NN) {
    return mul_diri<-DIR>(a);
  } else if constexpr (48 % NN == 0) {
    constexpr int j = mm * (48 / NN);
    constexpr double cd = cos48(j);
    constexpr double sd = DIR * sin48(j);
    const R c = (R)cd;
    const R s = (R)sd;
    return {a.x * c - a.y * s, a.x * s + a.y * c};
  } else {  // radix-9 and radix-18 steps
    constexpr double cd = cos_sin_frac(mm, NN, false);
    constexpr double sd = DIR * cos_sin_frac(mm, NN, true);
    const R c = (R)cd;
    const R s = (R)sd;
    return {a.x * c - a.y * s, a.x * s + a.y * c};
  }
}

template <int I, int N, typename F>
__device__ __forceinline__ void static_for(F &&f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>{});
    static_for<I + 1, N>(f);
  }
}

// In-register DFT of R points, x[k] <- sum_n x[n] exp(DIR 2 pi i n k / R).
template <int RR, int DIR, typename R>
struct DFT;

template <int DIR, typename R>
struct DFT<2, DIR, R> {
  __device__ __forceinline__ static void run(cpx<R> *x) {
    cpx<R> a = cadd(x[0], x[1]), b = csub(x[0], x[1]);
    x[0] = a;
    x[1] = b;
  }
};

template <int DIR, typename R>
struct DFT<3, DIR, R> {
  __device__ __forceinline__ static void run(cpx<R> *x) {
    const R h = (R)0.8660254037844386;  // sqrt(3)/2
    cpx<R> t1 = cadd(x[1], x[2]);
    cpx<R> d = csub(x[1], x[2]);
    cpx<R> t2 = mul_diri<DIR>(cscale(d, h));
    cpx<R> m = {x[0].x - (R)0.5 * t1.x, x[0].y - (R)0.5 * t1.y};
    x[0] = cadd(x[0], t1);
    x[1] = cadd(m, t2);
    x[2] = csub(m, t2);
  }
};

template <int DIR, typename R>
struct DFT<4, DIR, R> {
  __device__ __forceinline__ static void run(cpx<R> *x) {
    cpx<R> a0 = cadd(x[0], x[2]), a1 = csub(x[0], x[2]);
    cpx<R> a2 = cadd(x[1], x[3]), a3 = mul_diri<DIR>(csub(x[1], x[3]));
    x[0] = cadd(a0, a2);
    x[2] = csub(a0, a2);
    x[1] = cadd(a1, a3);
    x[3] = csub(a1, a3);
  }
};

// Five points: with t1 = x1 + x4, t2 = x2 + x3, t3 = x1 - x4, t4 = x2 - x3,
// X1,4 = x0 + c1 t1 + c2 t2 +- DIR i (s1 t3 + s2 t4) and
// X2,3 = x0 + c2 t1 + c1 t2 +- DIR i (s2 t3 - s1 t4), c_j + i s_j = e^(2 pi i j / 5).
template <int DIR, typename R>
struct DFT<5, DIR, R> {
  __device__ __forceinline__ static void run(cpx<R> *x) {
    constexpr double c1 = cos_sin_frac(1, 5, false), s1 = cos_sin_frac(1, 5, true);
    constexpr double c2 = cos_sin_frac(2, 5, false), s2 = cos_sin_frac(2, 5, true);
    const cpx<R> t1 = cadd(x[1], x[4]), t2 = cadd(x[2], x[3]), t3 = csub(x[1], x[4]), t4 = csub(x[2], x[3]);
    const cpx<R> a1 = {x[0].x + (R)c1 * t1.x + (R)c2 * t2.x, x[0].y + (R)c1 * t1.y + (R)c2 * t2.y};
    const cpx<R> a2 = {x[0].x + (R)c2 * t1.x + (R)c1 * t2.x, x[0].y + (R)c2 * t1.y + (R)c1 * t2.y};
    const cpx<R> b1 = mul_diri<DIR>(cpx<R>{(R)s1 * t3.x + (R)s2 * t4.x, (R)s1 * t3.y + (R)s2 * t4.y});
    const cpx<R> b2 = mul_diri<DIR>(cpx<R>{(R)s2 * t3.x - (R)s1 * t4.x, (R)s2 * t3.y - (R)s1 * t4.y});
    x[0] = cadd(x[0], cadd(t1, t2));
    x[1] = cadd(a1, b1);
    x[4] = csub(a1, b1);
    x[2] = cadd(a2, b2);
    x[3] = csub(a2, b2);
  }
};

// Composite RR = A * B, A in {4, 2, 3}:  n = B n1 + n2, k = k1 + A k2,
// X[k1 + A k2] = sum_n2 W_RR^(n2 k1) W_B^(n2 k2) [sum_n1 x[B n1 + n2] W_A^(n1 k1)].
template <int RR, int DIR, typename R>
struct DFT {
  static constexpr int A = (RR % 4 == 0) ? 4 : ((RR % 2 == 0) ? 2 : 3);
  static constexpr int B = RR / A;
  __device__ __forceinline__ static void run(cpx<R> *x) {
    cpx<R> y[B][A];
    static_for<0, B>([&](auto n2c) {
      constexpr int n2 = decltype(n2c)::value;
      cpx<R> t[A];
#pragma unroll
      for (int n1 = 0; n1 < A; ++n1) t[n1] = x[B * n1 + n2];
      DFT<A, DIR, R>::run(t);
      static_for<0, A>([&](auto k1c) {
        constexpr int k1 = decltype(k1c)::value;
        y[n2][k1] = twc<n2 * k1, RR, DIR>(t[k1]);
      });
    });
#pragma unroll
    for (int k1 = 0; k1 < A; ++k1) {
      cpx<R> t[B];
#pragma unroll
      for (int n2 = 0; n2 < B; ++n2) t[n2] = y[n2][k1];
      DFT<B, DIR, R>::run(t);
#pragma unroll
      for (int k2 = 0; k2 < B; ++k2) x[k1 + A * k2] = t[k2];
    }
  }
};

// ---- pass plan ----------------------------------------------------------
// After the radix-E first pass (in registers) the remaining factor T = N / E
// is split into radix-4 passes (and one radix-2 pass if T is an odd power of
// two).  Teams take radix-8 passes first where that keeps enough of the
// team busy: teams of 128 threads and more with E >= 6, whose radix-8 passes
// keep three quarters of the threads busy or more (512 threads, E = 6: 8, 8, 8
// instead of 4, 4, 4, 4, 2, 14% faster at 3072 points in FP32; the batch of
// tiles 4% faster), and teams of 1024 threads (8, 8, 4, 4: one LDS round trip
// fewer, 3% faster at 2048 points in FP64).  With E = 3 at 256 or 512 threads
// the fewer, larger butterflies measured slower.  Every later pass goes
// through LDS, its N / R butterflies spread over the T threads of the team.
__host__ __device__ constexpr int pass_radix(int T, int E, int rem) {
  return ((T >= 1024 || (T >= 128 && E >= 6)) && rem % 8 == 0 && rem != 16) ? 8 : ((rem % 4 == 0) ? 4 : 2);
}
__host__ __device__ constexpr int later_radix(int T, int E, int p) {  // p >= 1
  int rem = T;
  for (int i = 1; i < p; ++i) rem /= pass_radix(T, E, rem);
  return pass_radix(T, E, rem);
}
__host__ __device__ constexpr int num_passes(int T, int E) {
  int n = 1, rem = T;
  while (rem > 1) {
    rem /= pass_radix(T, E, rem);
    ++n;
  }
  return n;
}

// LDS index of element i of a transform buffer.  Unpadded: with 16-byte
// (FP64) or 8-byte (FP32) elements the Stockham access patterns measured
// faster without pad slots than with one slot every 16 elements.
__device__ __forceinline__ int lpad(int i) { return i; }
__host__ __device__ constexpr int lds_len(int N) { return N; }

// Team FFT of N = T * E points (unnormalised, sign DIR).  On entry thread t
// holds element t + T*r in v[r].  The first pass is a radix-E butterfly in
// registers; later passes exchange through LDS.  NBUF = 2 ping-pongs between
// buf0 and buf1 (one barrier per pass); NBUF = 1 works in place in buf0 (two
// barriers per pass).  The barriers are team_sync<T>: block barriers for
// teams spanning wavefronts, wavefront-level ordering for teams inside one.
// Returns the buffer holding the transform in natural order (lpad-indexed);
// the final barrier is included, so every thread of the team may read any
// element.  tw: the pass-ordered twiddle table of this (N, E).  Every thread
// of the team must call it (of the block, for teams spanning wavefronts).
// Pass-ordered twiddles: the later passes p = 1 .. NP-1 of a team FFT with
// first-pass radix E read W_N^(r k step_p) for r = 1 .. R_p-1 and
// k = 0 .. Ns_p-1 (Ns_p = E R_1 ... R_(p-1), step_p = N / (Ns_p R_p)).  The
// host stores them at Ns_p - E + (r-1) Ns_p + k (N - E entries), so a lane's
// consecutive k read adjacent words instead of a stride of r step_p.  Each
// transform length keeps one table per candidate E, slot tw_slot(E).
// Slots: E in {2, 3, 9, 10, 15} -> 0, {4, 6, 18} -> 1, {8, 12} -> 2 (a length
// uses at most one E of each group).
// Slot 3 holds the natural table W_N^m, m < N (the permuted-layout forms
// below).
constexpr int kTwSlots = 4;
constexpr int kTwNatural = 3;
__host__ __device__ constexpr int tw_slot(int E) {
  return (E == 2 || E == 3 || E == 9 || E == 10 || E == 15) ? 0 : ((E == 4 || E == 6 || E == 18) ? 1 : 2);
}

// Last pass of a team FFT of N = E T points: radix R, NB = N / R butterflies,
// IT per thread.  Butterfly j = t + T it of that pass owns the elements
// j + NB r, r < R, of the natural-order result (its output base is j).
template <int N, int E>
struct LastPass {
  static constexpr int T = N / E;
  static constexpr int NP = num_passes(T, E);
  static constexpr int R = later_radix(T, E, NP - 1);
  static constexpr int NB = N / R;
  static constexpr int IT = (NB + T - 1) / T;
};
// Registers of the last pass's butterflies: [it][r] holds element j + NB r.
template <typename R, int N, int E>
using LastRegs = cpx<R>[LastPass<N, E>::IT][LastPass<N, E>::R];

// LDS ordering inside one wavefront: its LDS operations complete in issue
// order, so a compiler barrier is all a wavefront-private exchange needs.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
// The synchronisation of a team of T threads around its LDS exchanges: a
// team of at most 64 threads lies inside one wavefront (teams are aligned)
// and owns its buffers, so it orders them without a block barrier; larger
// teams span wavefronts and take one.
template <int T>
__device__ __forceinline__ void team_sync() {
  if constexpr (T <= 64) wave_lds_sync();
  else __syncthreads();
}

// Shared body of the two forward-order forms.  KEEP = false: the last pass
// writes LDS and a final barrier follows (team_fft).  KEEP = true: the last
// pass leaves butterfly j's outputs in o[it][r] (element j + NB r) and no
// barrier follows (team_fft_keep); the next transform's first barrier
// protects the buffers.
template <typename R, int N, int E, int NBUF, int DIR, bool KEEP>
__device__ __forceinline__ cpx<R> *team_fft_impl(cpx<R> (&v)[E], cpx<R> *buf0, cpx<R> *buf1,
                                                 const cpx<R> *__restrict__ tw, int t,
                                                 cpx<R> (*o)[LastPass<N, E>::R]) {
  constexpr int T = N / E;
  constexpr int NP = num_passes(T, E);
  static_assert(NP >= 2, "team FFT needs at least two passes");
  // Make the lane index opaque (an empty asm statement, no instruction): the
  // per-pass LDS and twiddle addresses derived from it are then recomputed at
  // each transform instead of being hoisted out of the callers' loops and
  // kept live for the whole kernel.
  asm volatile("" : "+v"(t));
  DFT<E, DIR, R>::run(v);
  team_sync<T>();  // readers of the previous transform's result are done
#pragma unroll
  for (int r = 0; r < E; ++r) buf0[lpad(t * E + r)] = v[r];
  cpx<R> *in = buf0;
  cpx<R> *out = NBUF == 2 ? buf1 : buf0;
  static_for<1, NP>([&](auto pc) {
    constexpr int p = decltype(pc)::value;
    constexpr int Rp = later_radix(T, E, p);
    constexpr int nb = N / Rp;
    constexpr int IT = (nb + T - 1) / T;
    constexpr int Ns = [] {
      int ns = E;
      for (int i = 1; i < p; ++i) ns *= later_radix(T, E, i);
      return ns;
    }();
    constexpr bool to_regs = KEEP && p == NP - 1;
    team_sync<T>();
    cpx<R> w[IT][Rp];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int j = t + T * it;
      if (j < nb) {
#pragma unroll
        for (int r = 0; r < Rp; ++r) w[it][r] = in[lpad(j + r * nb)];
      }
    }
    if constexpr (NBUF == 1 && !to_regs) team_sync<T>();
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int j = t + T * it;
      if (j < nb) {
        const int k = j % Ns;
#pragma unroll
        for (int r = 1; r < Rp; ++r) {
          cpx<R> tr = tw[Ns - E + (r - 1) * Ns + k];
          if constexpr (DIR > 0) tr.y = -tr.y;
          w[it][r] = cmul(w[it][r], tr);
        }
        DFT<Rp, DIR, R>::run(w[it]);
        if constexpr (to_regs) {
#pragma unroll
          for (int r = 0; r < Rp; ++r) o[it][r] = w[it][r];  // base = j in the last pass
        } else {
          const int base = (j / Ns) * Ns * Rp + k;
#pragma unroll
          for (int r = 0; r < Rp; ++r) out[lpad(base + r * Ns)] = w[it][r];
        }
      }
    }
    if constexpr (NBUF == 2) {
      cpx<R> *tmp = in;
      in = out;
      out = tmp;
    }
  });
  if constexpr (!KEEP) team_sync<T>();
  return in;
}

template <typename R, int N, int E, int NBUF, int DIR>
__device__ __forceinline__ cpx<R> *team_fft(cpx<R> (&v)[E], cpx<R> *buf0, cpx<R> *buf1,
                                            const cpx<R> *__restrict__ tw, int t) {
  return team_fft_impl<R, N, E, NBUF, DIR, false>(v, buf0, buf1, tw, t, nullptr);
}

// Team FFT whose result stays in registers in the last pass's layout:
// o[it][r] = X[j + NB r] for butterfly j = t + T it < NB (LastPass<N, E>);
// o is unset where j >= NB.  In: as team_fft.
template <typename R, int N, int E, int NBUF, int DIR>
__device__ __forceinline__ void team_fft_keep(cpx<R> (&v)[E], cpx<R> *buf0, cpx<R> *buf1,
                                              const cpx<R> *__restrict__ tw, int t,
                                              LastRegs<R, N, E> &o) {
  team_fft_impl<R, N, E, NBUF, DIR, true>(v, buf0, buf1, tw, t, o);
}

// Transposed team FFT: the same passes in reverse order, each with its
// gather and scatter exchanged and its twiddles applied after the butterfly
// (the transpose of the algorithm above; the DFT matrix is symmetric, so it
// computes the same transform from the same twiddle table).  In: x[it][r] =
// x[j + NB r] for butterfly j = t + T it < NB of LastPass<N, E> (unused where
// j >= NB), the layout in which the caller loads it; out: v[r] = X[t + T r],
// the layout of team_fft's input.  No LDS readout: the last (radix-E) step
// runs in registers.  Every thread of the team must call it (of the block, for
// teams spanning wavefronts).
template <typename R, int N, int E, int NBUF, int DIR>
__device__ __forceinline__ void team_fft_t(LastRegs<R, N, E> &x, cpx<R> (&v)[E], cpx<R> *buf0, cpx<R> *buf1,
                                           const cpx<R> *__restrict__ tw, int t) {
  constexpr int T = N / E;
  constexpr int NP = num_passes(T, E);
  static_assert(NP >= 2, "team FFT needs at least two passes");
  asm volatile("" : "+v"(t));
  cpx<R> *in = buf0;
  cpx<R> *out = buf0;
  team_sync<T>();  // readers of the previous transform's buffers are done
  static_for<1, NP>([&](auto qc) {
    constexpr int p = NP - decltype(qc)::value;  // NP - 1 down to 1
    constexpr int Rp = later_radix(T, E, p);
    constexpr int nb = N / Rp;
    constexpr int IT = (nb + T - 1) / T;
    constexpr int Ns = [] {
      int ns = E;
      for (int i = 1; i < p; ++i) ns *= later_radix(T, E, i);
      return ns;
    }();
    constexpr bool from_regs = p == NP - 1;
    cpx<R> w[IT][Rp];
    if constexpr (!from_regs) {
      team_sync<T>();
#pragma unroll
      for (int it = 0; it < IT; ++it) {
        const int j = t + T * it;
        if (j < nb) {
          const int base = (j / Ns) * Ns * Rp + j % Ns;
#pragma unroll
          for (int r = 0; r < Rp; ++r) w[it][r] = in[lpad(base + r * Ns)];
        }
      }
      if constexpr (NBUF == 1) team_sync<T>();
    }
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int j = t + T * it;
      if (j < nb) {
        if constexpr (from_regs) {
#pragma unroll
          for (int r = 0; r < Rp; ++r) w[it][r] = x[it][r];
        }
        const int k = j % Ns;
        DFT<Rp, DIR, R>::run(w[it]);
#pragma unroll
        for (int r = 1; r < Rp; ++r) {
          cpx<R> tr = tw[Ns - E + (r - 1) * Ns + k];
          if constexpr (DIR > 0) tr.y = -tr.y;
          w[it][r] = cmul(w[it][r], tr);
        }
#pragma unroll
        for (int r = 0; r < Rp; ++r) out[lpad(j + r * nb)] = w[it][r];
      }
    }
    in = out;
    if constexpr (NBUF == 2) out = (out == buf0) ? buf1 : buf0;
  });
  team_sync<T>();
#pragma unroll
  for (int r = 0; r < E; ++r) v[r] = in[lpad(t * E + r)];
  DFT<E, DIR, R>::run(v);
}

// Register layouts on the HBM side of a transform.  LAST: the last pass's
// butterfly layout ([it][r] = element t + T it + NB r, live where
// t + T it < NB), used by team_fft_t (input) and team_fft_keep (output);
// otherwise the team layout ([0][r] = element t + T r).
template <int N, int E, bool LAST>
struct HbmLayout {
  static constexpr int T = N / E;
  static constexpr int IT = LAST ? LastPass<N, E>::IT : 1;
  static constexpr int R = LAST ? LastPass<N, E>::R : E;
  static constexpr int STRIDE = LAST ? LastPass<N, E>::NB : T;
  __device__ __forceinline__ static bool live(int t, int it) { return !LAST || t + T * it < LastPass<N, E>::NB; }
  __device__ __forceinline__ static int elem(int t, int it, int r) { return t + T * it + STRIDE * r; }
};
template <typename R, int N, int E, bool LAST>
using HbmRegs = cpx<R>[HbmLayout<N, E, LAST>::IT][HbmLayout<N, E, LAST>::R];

// x in the HBM-side layout -> v[r] = X[t + T r].
template <typename R, int N, int E, int NBUF, int DIR, bool LAST>
__device__ __forceinline__ void fft_in(HbmRegs<R, N, E, LAST> &x, cpx<R> (&v)[E], cpx<R> *buf0, cpx<R> *buf1,
                                       const cpx<R> *__restrict__ tw, int t) {
  if constexpr (LAST) {
    team_fft_t<R, N, E, NBUF, DIR>(x, v, buf0, buf1, tw, t);
  } else {
#pragma unroll
    for (int r = 0; r < E; ++r) v[r] = x[0][r];
    const cpx<R> *res = team_fft<R, N, E, NBUF, DIR>(v, buf0, buf1, tw, t);
#pragma unroll
    for (int r = 0; r < E; ++r) v[r] = res[lpad(t + (N / E) * r)];
  }
}

// ---- permuted-layout transforms --------------------------------------------
// For a team of T = 64 W threads (W wavefronts, W a power of two up to 16)
// and N = E T points.  perm_ifft takes v[r] = x[t + T r] (natural order) and
// leaves the transform in a permuted order; perm_fft takes that permuted
// order and returns natural order.  Between the two, pointwise products do
// not care where a point sits, so neither form spends an LDS pass on
// reordering, and only the stages whose butterflies span wavefronts meet at
// block barriers.  With t = 64 w + l (wavefront w, lane l) and three digits
// n = l + 64 w + 64 W r, k = k_a + E k_b + E W k_c, the inverse transform is
//   a  = DFT_E over r (registers), times W_N^(64 w k_a);
//   b  = DFT_W over w (wavefronts: radix-4/2 decimation-in-frequency stages
//        through LDS, one barrier each; wave w ends up holding k_b =
//        bitrev(w)), times W_N^(l (k_a + E k_b));
//   X  = DFT_64 over l (lanes) for each (k_a, k_b): six radix-2
//        decimation-in-frequency stages whose partners l ^ h are exchanged
//        across lanes (DPP permutes, ds_bpermute), no LDS storage, no
//        barrier; lane l ends up holding k_c = bitrev6(l).
// Thread t then holds in v[s] the point s + E bitrev(w) + E W bitrev6(l).  perm_fft is
// the same algorithm transposed (the DFT matrix is symmetric): the lane DFT
// first, the twiddles, the wavefront stages as decimation-in-time, the
// register DFT last.  Twiddles come from the natural table W_N^m (forward
// sign; conjugated for DIR > 0).


template <int DIR, typename R>
__device__ __forceinline__ cpx<R> twn(const cpx<R> *tw, int m) {
  cpx<R> w = tw[m];
  if constexpr (DIR > 0) w.y = -w.y;
  return w;
}

__host__ __device__ constexpr int ilog2c(int x) { return x <= 1 ? 0 : 1 + ilog2c(x / 2); }

// Lane l ^ H's copy of a 32-bit value: DPP within rows of 16 lanes (H <= 8:
// quad permutes, the half-row mirror followed by a quad reversal, a row
// rotation by 8), ds_bpermute across rows.
template <int H>
__device__ __forceinline__ int lane_xor(int v) {
  if constexpr (H == 1) return __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xF, 0xF, false);  // quad_perm [1,0,3,2]
  else if constexpr (H == 2) return __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xF, 0xF, false);  // quad_perm [2,3,0,1]
  else if constexpr (H == 4) {
    const int m = __builtin_amdgcn_update_dpp(0, v, 0x141, 0xF, 0xF, false);  // row_half_mirror: i -> 7 - i
    return __builtin_amdgcn_update_dpp(0, m, 0x1B, 0xF, 0xF, false);          // quad_perm [3,2,1,0]
  } else if constexpr (H == 8) return __builtin_amdgcn_update_dpp(0, v, 0x128, 0xF, 0xF, false);  // row_ror:8
  else return __shfl_xor(v, H, 64);
}
template <int H>
__device__ __forceinline__ double lane_xor(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = lane_xor<H>((int)(unsigned)b), hi = lane_xor<H>((int)(unsigned)(b >> 32));
  return __longlong_as_double(((long long)(unsigned)hi << 32) | (unsigned)lo);
}
template <int H>
__device__ __forceinline__ float lane_xor(float v) {
  return __int_as_float(lane_xor<H>(__float_as_int(v)));
}

// 64-point DFT over the lanes of one wavefront for each of its E sequences,
// by radix-2 stages whose partners are exchanged across lanes (lane_xor):
// DIF: natural order in, bit-reversed out (lane l holds X[bitrev6(l)]); DIT
// (the transpose): bit-reversed in, natural out.  Stage h's factor
// W_2h^(l mod h) multiplies the upper lane's difference (DIF) or its own
// value before the exchange (DIT).
template <typename R, int N, int E, int DIR, bool DIF>
__device__ __forceinline__ void wave_dft64_x(cpx<R> (&v)[E], const cpx<R> *__restrict__ tw, int l) {
  static_for<0, 6>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    constexpr int h = DIF ? (32 >> i) : (1 << i);
    const bool B = (l & h) != 0;
    const R sg = B ? (R)-1 : (R)1;
    cpx<R> ws = {(R)1, (R)0};
    if constexpr (h > 1) {
      const cpx<R> wt = twn<DIR>(tw, (l & (h - 1)) * (N / (2 * h)));
      if (B) ws = wt;
    }
#pragma unroll
    for (int q = 0; q < E; ++q) {
      if constexpr (DIF) {
        const cpx<R> p = {lane_xor<h>(v[q].x), lane_xor<h>(v[q].y)};
        const cpx<R> d = {p.x + sg * v[q].x, p.y + sg * v[q].y};
        v[q] = h > 1 ? cmul(d, ws) : d;
      } else {
        const cpx<R> c = h > 1 ? cmul(v[q], ws) : v[q];
        const cpx<R> p = {lane_xor<h>(c.x), lane_xor<h>(c.y)};
        v[q] = {p.x + sg * c.x, p.y + sg * c.y};
      }
    }
  });
}

// Wavefront stages of the W-point DFT: spans in wavefronts, from the top,
// radix 4 (spans hw, hw / 2) while two bits remain, else radix 2.
__host__ __device__ constexpr int xw_stages(int W) {
  int n = 0;
  for (int hw = W / 2; hw >= 1; hw = hw >= 2 ? hw / 4 : hw / 2) ++n;
  return n;
}
__host__ __device__ constexpr int xw_span(int W, int i) {  // top span of decimation-in-frequency stage i
  int hw = W / 2;
  for (int k = 0; k < i; ++k) hw = hw >= 2 ? hw / 4 : hw / 2;
  return hw;
}

// One wavefront stage of the decimation-in-frequency DFT over w (FWD) or of
// its transpose (decimation in time), on every register: v goes out through
// buf (layout [E][T]), one block barrier, and the partners come back.  HW:
// the stage's top span in wavefronts (radix 4 for HW >= 2: spans HW, HW / 2).
// The butterfly's position bits are wavefront-uniform, so its branches are.
template <typename R, int T, int E, int DIR, int HW, bool DIF>
__device__ __forceinline__ void xw_stage(cpx<R> (&v)[E], cpx<R> *buf, const cpx<R> *__restrict__ tw, int t, int w) {
  constexpr int N = T * E;
#pragma unroll
  for (int q = 0; q < E; ++q) buf[q * T + t] = v[q];
  __syncthreads();
  if constexpr (HW == 1) {
    const bool B = (w & 1) != 0;
    const int tp = t ^ 64;
    // W_2^0 = 1: the one radix-2 stage with span one wavefront has no twiddle
#pragma unroll
    for (int q = 0; q < E; ++q) {
      const cpx<R> p = buf[q * T + tp];
      v[q] = B ? csub(p, v[q]) : cadd(v[q], p);
    }
  } else {
    constexpr int H2 = HW / 2;
    const int t0 = t & ~(96 * HW);
    const int w0 = w & ~(HW | H2);
    const bool B1 = (w & HW) != 0, B0 = (w & H2) != 0;
    const cpx<R> w1 = twn<DIR>(tw, (w0 % HW) * (N / (2 * HW)));
    const cpx<R> w2 = twn<DIR>(tw, (w0 % H2) * (N / HW));
#pragma unroll
    for (int q = 0; q < E; ++q) {
      const cpx<R> i0 = buf[q * T + t0], i1 = buf[q * T + t0 + 32 * HW];
      const cpx<R> i2 = buf[q * T + t0 + 64 * HW], i3 = buf[q * T + t0 + 96 * HW];
      if constexpr (DIF) {
        // positions t0 + {0, 32 HW, 64 HW, 96 HW} hold a0, a1, b0, b1
        const cpx<R> x0 = B1 ? cmul(csub(i0, i2), w1) : cadd(i0, i2);
        const cpx<R> x1 = B1 ? mul_diri<DIR>(cmul(csub(i1, i3), w1)) : cadd(i1, i3);
        v[q] = B0 ? cmul(csub(x0, x1), w2) : cadd(x0, x1);
      } else {
        const cpx<R> m1 = cmul(i1, w2), m3 = cmul(i3, w2);
        const cpx<R> c = B0 ? csub(i0, m1) : cadd(i0, m1);
        const cpx<R> d = B0 ? csub(i2, m3) : cadd(i2, m3);
        const cpx<R> fd = B0 ? mul_diri<DIR>(cmul(d, w1)) : cmul(d, w1);
        v[q] = B1 ? csub(c, fd) : cadd(c, fd);
      }
    }
  }
}

// x[t + T r] in v[r] -> v[s] = X[s + E bitrev(w) + E W bitrev6(l)] (sign DIR).  b0, b1:
// the team's two LDS buffers of N entries; tw: the natural table.  Opens
// with a block barrier when W > 1 (earlier readers of both buffers are done);
// closes without one.  Every thread of the block must call it.
template <typename R, int T, int E, int DIR>
__device__ __forceinline__ void perm_ifft(cpx<R> (&v)[E], cpx<R> *b0, cpx<R> *b1, const cpx<R> *__restrict__ tw,
                                          int t) {
  constexpr int N = T * E, W = T / 64, NS = xw_stages(W);
  static_assert(T % 64 == 0 && W <= 16, "team of whole wavefronts");
  const int w = __builtin_amdgcn_readfirstlane(t >> 6), l = t & 63;
  DFT<E, DIR, R>::run(v);
#pragma unroll
  for (int q = 1; q < E; ++q) v[q] = cmul(v[q], twn<DIR>(tw, 64 * w * q));
  if constexpr (W > 1) {
    __syncthreads();
    static_for<0, NS>([&](auto ic) {
      constexpr int i = decltype(ic)::value;
      xw_stage<R, T, E, DIR, xw_span(W, i), true>(v, i % 2 == 0 ? b0 : b1, tw, t, w);
    });
  }
  const int kb = W > 1 ? (int)(__builtin_bitreverse32((unsigned)w) >> (32 - ilog2c(W))) : 0;
#pragma unroll
  for (int q = 0; q < E; ++q)
    if (q > 0 || kb > 0) v[q] = cmul(v[q], twn<DIR>(tw, l * (q + E * kb)));
  wave_dft64_x<R, N, E, DIR, true>(v, tw, l);
}

// v[s] = x[s + E bitrev(w) + E W bitrev6(l)] -> X[t + T r] in natural order in the
// returned LDS buffer (sign DIR), after a closing block barrier (every thread
// may read any element; W = 1: the team is one wavefront, which the closing
// wavefront ordering covers).  OPEN: open with a block barrier (omit only
// where one since the last read of the buffers precedes the call).
template <typename R, int T, int E, int DIR, bool OPEN = true>
__device__ __forceinline__ const cpx<R> *perm_fft(cpx<R> (&v)[E], cpx<R> *b0, cpx<R> *b1,
                                                  const cpx<R> *__restrict__ tw, int t) {
  constexpr int N = T * E, W = T / 64, NS = xw_stages(W);
  static_assert(T % 64 == 0 && W <= 16, "team of whole wavefronts");
  const int w = __builtin_amdgcn_readfirstlane(t >> 6), l = t & 63;
  if constexpr (OPEN && W > 1) __syncthreads();
  wave_dft64_x<R, N, E, DIR, false>(v, tw, l);
  const int kb = W > 1 ? (int)(__builtin_bitreverse32((unsigned)w) >> (32 - ilog2c(W))) : 0;
#pragma unroll
  for (int q = 0; q < E; ++q)
    if (q > 0 || kb > 0) v[q] = cmul(v[q], twn<DIR>(tw, l * (q + E * kb)));
  // transposed wavefront stages in reverse order; the first writes b1 (other
  // wavefronts may still read their regions of b0)
  static_for<0, NS>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    xw_stage<R, T, E, DIR, xw_span(W, NS - 1 - i), false>(v, i % 2 == 0 ? b1 : b0, tw, t, w);
  });
#pragma unroll
  for (int q = 1; q < E; ++q) v[q] = cmul(v[q], twn<DIR>(tw, 64 * w * q));
  DFT<E, DIR, R>::run(v);
  cpx<R> *out = NS % 2 == 1 ? b0 : b1;  // not read by the last stage
#pragma unroll
  for (int r = 0; r < E; ++r) out[t + T * r] = v[r];
  if constexpr (W > 1) __syncthreads();
  else wave_lds_sync();
  return out;
}

}  // namespace zk
