// zk_kernels.hpp -- row-pass and column-pass kernels of the HOS pipeline.
//
// Data layouts (all device memory carved from the caller's workspace):
//   base spectrum   complex<double> [nx/2 / CBB][ny][CBB] with CBB = 1, i.e.
//                   column-major: column kx (0 <= kx < nx/2; the kx = nx/2
//                   Nyquist column is not stored) holds its ny ky modes
//                   contiguously, index b = ky mode mod ny (b = ny/2 is the
//                   Nyquist row, kept 0).
//   mixed field     complex<real> [nx/2 / CB][rows][CB]: y physical (rows =
//                   3ny/2 padded, or ny for the base transforms), kx spectral.
//   caller fields   double [ny][nx] row-major.
// A row team of T threads owns one row, a column team one kx column; T and
// the first-pass radix E are template parameters (T * E = transform length).
// Every index below stays inside these arrays when the host launches exactly
// rows / TPB x nprog row blocks and ncols / TPB x ntask column blocks
// (checked on the host).
#pragma once
#include "zk_fft.hpp"
#include "zk_program.hpp"
#include "zk_row_shapes.hpp"

namespace zk {

constexpr int CBB = 1;  // tile width of base spectra: 1 = column-major, each column contiguous

template <typename real>
struct MixTile {
  static constexpr int CB = sizeof(real) == 8 ? 4 : 8;  // 64 B segments
};

template <typename real>
struct RowArgs {
  const RowOp *ops;
  const RowProg *progs;
  int prog0;
  cpx<real> *mix;
  long long mix_stride;  // elements between mixed fields
  int rows;              // rows of the mixed fields of this pass
  int nx;                // base-grid row length (physical fields)
  const double *pin0, *pin1, *pin2;  // OP_LDP slots 0..2
  double *pout0, *pout1;             // OP_STP slots 0..1
  const cpx<real> *tw;    // kTwSlots twiddle tables (pass-ordered, natural) of the row FFT length N
  double kx_scale;        // 2 pi / Lx
  const float *colmax;    // [mixed field][nx/2]: per-column max |value| written by the lifts
};


template <typename real>
struct ColArgs {
  const ColTask *tasks;
  int task0;
  const ColOut *outs;
  const ColTerm *terms;
  cpx<real> *mix;
  long long mix_stride;
  int rows;  // column FFT length (3ny/2 or ny)
  cpx<double> *base;
  long long base_stride;
  int ny, nx;
  const cpx<real> *tw;  // kTwSlots twiddle tables (pass-ordered, natural) of the column FFT length
  double kx_scale, ky_scale;
  double depth;   // <= 0: deep water
  double inv_kc;  // 1 / kc of the taper
  int taper_on;
  float *colmax;  // [mixed field][nx/2]: max |value| of each lifted column
  // per band element, base-spectrum layout: G0 = |k| tanh(|k| d) (read only
  // at finite depth; deep water has G0 = |k|) and the taper exp(-(|k|/kc)^8)
  // (read only while the taper is on, by tasks that fold); |k| itself is
  // computed in the kernel
  const double *sym_g0, *sym_tp;
  const double *filt_x, *filt_y;  // separable state filter factors
  const double *ifsym;            // kIfCoefs per band element (base layout), or null
  const double *layer_y;          // depths of the current chunk of layers (kMaxChunkLayers)
};

// ---- register-set dispatch (keeps every register array statically indexed)
template <typename F>
__device__ __forceinline__ void with_in(int s, F &&f) {  // u, v, A
  switch (s) {
    case 0: f(std::integral_constant<int, 0>{}); break;
    case 1: f(std::integral_constant<int, 1>{}); break;
    case 2: f(std::integral_constant<int, 2>{}); break;
    default: break;
  }
}
template <typename F>
__device__ __forceinline__ void with_out(int s, F &&f) {  // o0, o1, o2
  switch (s) {
    case 3: f(std::integral_constant<int, 3>{}); break;
    case 4: f(std::integral_constant<int, 4>{}); break;
    case 5: f(std::integral_constant<int, 5>{}); break;
    default: break;
  }
}
template <typename F>
__device__ __forceinline__ void with_any(int s, F &&f) {
  switch (s) {
    case 0: f(std::integral_constant<int, 0>{}); break;
    case 1: f(std::integral_constant<int, 1>{}); break;
    case 2: f(std::integral_constant<int, 2>{}); break;
    case 3: f(std::integral_constant<int, 3>{}); break;
    case 4: f(std::integral_constant<int, 4>{}); break;
    case 5: f(std::integral_constant<int, 5>{}); break;
    default: break;
  }
}

// element offsets inside one field (fields hold < 2^31 elements)
template <typename real>
__device__ __forceinline__ int mix_index(int kx, int y, int rows) {
  constexpr int CB = MixTile<real>::CB;
  return ((kx / CB) * rows + y) * CB + (kx % CB);
}
__device__ __forceinline__ int base_index(int kx, int b, int ny) {
  return ((kx / CBB) * ny + b) * CBB + (kx % CBB);
}

// XCD-aware block placement.  Consecutive block indices are dispatched
// round-robin over the 8 XCDs, each with its own L2.  Units (rows or groups
// of columns) that share 128-byte lines of a tiled field -- `per` units --
// are given block indices that are congruent mod 8, so they run on one XCD
// and share its L2 instead of each XCD fetching the line.  Identity when the
// unit count does not split evenly.
__device__ __forceinline__ int xcd_unit(int b, int nunits, int per) {
  if (per <= 1 || nunits % (8 * per) != 0) return b;
  const int x = b & 7, slot = b >> 3;
  return ((slot / per) * 8 + x) * per + (slot % per);
}

// Max of a non-negative float over the 64 lanes of a wavefront, returned
// to every lane: DPP row shifts build each 16-lane row's max in its last
// lane, two row broadcasts carry it to lane 63, and a readlane hands it out.
// Non-negative floats order like their bit patterns, so the max runs on
// unsigned words; lanes whose DPP source lies outside the row read 0.
__device__ __forceinline__ float wave_max(float x) {
  unsigned v = __float_as_uint(x);
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, false));  // row_shr:1
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, false));  // row_shr:2
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, false));  // row_shr:4
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, false));  // row_shr:8
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false));  // row_bcast:15
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false));  // row_bcast:31
  return __uint_as_float((unsigned)__builtin_amdgcn_readlane((int)v, 63));
}

// Max over one team of T threads (non-negative values).  Teams of fewer than
// 64 threads sit inside one wavefront and reduce with lane shuffles, a full
// wavefront with wave_max; larger teams (one per block) add an LDS step
// across their wavefronts.  red: >= one float per wavefront of the block.  Every
// thread of the block must call it.
template <int T>
__device__ __forceinline__ float team_max(float v, float *red) {
  constexpr int W = T < 64 ? T : 64;
  if constexpr (W == 64) {
    v = wave_max(v);
  } else {
#pragma unroll
    for (int o = W / 2; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
  }
  if constexpr (T > 64) {
    const int w0 = (threadIdx.x / T) * (T / 64);  // first wavefront of this team
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    v = red[w0];
#pragma unroll
    for (int k = 1; k < T / 64; ++k) v = fmaxf(v, red[w0 + k]);
  }
  return v;
}

// Max of two values over one team at once (same scheme as team_max).
// red: >= two floats per wavefront of the block.
template <int T>
__device__ __forceinline__ float2 team_max2(float a, float b, float *red) {
  constexpr int W = T < 64 ? T : 64;
  if constexpr (W == 64) {
    a = wave_max(a);
    b = wave_max(b);
  } else {
#pragma unroll
    for (int o = W / 2; o > 0; o >>= 1) {
      a = fmaxf(a, __shfl_xor(a, o, 64));
      b = fmaxf(b, __shfl_xor(b, o, 64));
    }
  }
  if constexpr (T > 64) {
    const int w0 = (threadIdx.x / T) * (T / 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) {
      red[2 * (threadIdx.x >> 6)] = a;
      red[2 * (threadIdx.x >> 6) + 1] = b;
    }
    __syncthreads();
    a = red[2 * w0];
    b = red[2 * w0 + 1];
#pragma unroll
    for (int k = 1; k < T / 64; ++k) {
      a = fmaxf(a, red[2 * (w0 + k)]);
      b = fmaxf(b, red[2 * (w0 + k) + 1]);
    }
  }
  return make_float2(a, b);
}

// Power-of-two scale s bringing a magnitude m to [1, 2), and 1/s, both exact:
// (2^-e, 2^e) with m in [2^e, 2^(e+1)).  For m = 0 the field is zero (below
// FP32's smallest magnitude) and the pair is (1, 0), so its half of a paired
// transform comes out exactly zero instead of carrying its partner's rounding.
__device__ __forceinline__ float2 pow2_scale(float m) {
  if (m == 0.f) return make_float2(1.0f, 0.0f);
  if (!(m > 0.f && m < 3.0e38f)) return make_float2(1.0f, 1.0f);
  const int e = ilogbf(m);
  return make_float2(ldexpf(1.0f, -e), ldexpf(1.0f, e));
}

// ---------------------------------------------------------------------------
// Shape constants of a team: T threads, E first-pass elements per thread.
// E % 3 == 0: a 3/2-padded transform of N = T E = 3n/2 points, whose n/2
// retained band slots are r < E/3 (positive) and r >= 2E/3 (negative);
// otherwise a base transform of N = n points, retained r < E/2 and r >= E/2.
// In both cases the band has K = (E/3 or E/2) * T = n/2 positive modes, and
// slot "first negative, t = 0" is the Nyquist mode (never stored).
// Whether a row team shape (T threads, E elements, default block of
// max(T, 256) threads) has the permuted-layout transforms: padded, whole
// wavefronts, and room for two LDS buffers per team (the twiddle table goes
// to LDS only if it fits beside them).
__host__ __device__ constexpr bool row_lanes_ok(int T, int E, bool padded, int real_bytes) {
  const int N = T * E, tpb = (T > 256 ? T : 256) / T;
  return padded && E % 5 != 0 && T % 64 == 0 && T <= 1024 && 2 * tpb * N * 2 * real_bytes <= 100 * 1024;
}

// Number of LD2 operations among the first i operations of compiled shape sh
// (at an LD2: its ordinal among the shape's LD2s).
constexpr int row_shape_ld2_ordinal(int sh, int i) {
  int n = 0;
  for (int k = 0; k < i; ++k) n += (kRowShapeOps[sh][k] & 255) == OP_LD2 ? 1 : 0;
  return n;
}
constexpr int row_shapes_max_ld2() {
  int m = 0;
  for (int sh = 0; sh < kRowShapes; ++sh) {
    const int n = row_shape_ld2_ordinal(sh, kRowShapeLen[sh]);
    m = n > m ? n : m;
  }
  return m;
}
constexpr int kRowShapeMaxLd2 = row_shapes_max_ld2();
// Column-maxima count from which compiled programs reduce them per block.
constexpr int kBlockMaximaCols = 1024;

// Padded row shapes whose kernels also hold every program shape of
// zk_row_shapes.hpp as straight-line code (the team shapes the autotuner
// picks for the large grids; the others interpret every program).
__host__ __device__ constexpr bool row_compiled_shapes(int T, int E, bool padded) {
  return padded && ((E == 3 && T >= 64 && T <= 1024) || (E == 6 && T >= 128 && T <= 512));
}

template <int T, int E, int BSZ = 0, bool PAD = (E % 3 == 0)>
struct Shape {
  static constexpr bool PADDED = PAD;
  static constexpr int N = T * E;
  static constexpr int KR = PADDED ? E / 3 : E / 2;    // positive slots
  static constexpr int NEG0 = PADDED ? 2 * E / 3 : E / 2;  // first negative slot
  static constexpr int QB = PADDED ? 2 * E / 3 : E;    // base-band elements per thread
  static constexpr int BS = BSZ ? BSZ : (T > 256 ? T : 256);  // threads per block (default max(T, 256))
  static constexpr int TPB = BS / T;                   // teams per block
  static constexpr int L = lds_len(N);
  // two LDS buffers per team when they fit comfortably beside the twiddle
  // table, else one (the permuted-layout forms, LANES, always take two)
  template <typename real, bool LANES = false>
  static constexpr int nbuf() {
    return LANES || (2 * TPB * L + N) * (int)sizeof(cpx<real>) <= 100 * 1024 ? 2 : 1;
  }
  template <typename real, bool LANES = false>
  static constexpr bool tw_in_lds() {
    return (nbuf<real, LANES>() * TPB * L + N) * (int)sizeof(cpx<real>) <= 100 * 1024;
  }
  // Padded row passes of whole-wavefront teams with two buffers can also run
  // their transforms in the permuted layout with lane-exchange butterflies
  // (perm_ifft / perm_fft); the caller picks the form at run time.
  template <typename real>
  static constexpr bool lanes_ok() {
    return row_lanes_ok(T, E, PADDED, (int)sizeof(real));
  }
};

// Field data goes through global-address-space pointers: global loads and
// stores (not flat ones, which also count against the LDS wait counter and
// would make every LDS wait of a transform wait for them too).
template <typename R>
struct Vec2 {
  typedef R T __attribute__((ext_vector_type(2)));
};
template <typename R>
__device__ __forceinline__ cpx<R> gload(const cpx<R> *p, long long i) {
  const typename Vec2<R>::T v = ((const __attribute__((address_space(1))) typename Vec2<R>::T *)p)[i];
  return {v.x, v.y};
}
template <typename R>
__device__ __forceinline__ void gstore(cpx<R> *p, long long i, cpx<R> c) {
  typename Vec2<R>::T v;
  v.x = c.x;
  v.y = c.y;
  ((__attribute__((address_space(1))) typename Vec2<R>::T *)p)[i] = v;
}
template <typename Tp>
__device__ __forceinline__ Tp gload1(const Tp *p, long long i) {
  return ((const __attribute__((address_space(1))) Tp *)p)[i];
}
template <typename Tp>
__device__ __forceinline__ void gstore1(Tp *p, long long i, Tp v) {
  ((__attribute__((address_space(1))) Tp *)p)[i] = v;
}

// Schedule records (programs, ops, tasks, outputs, terms) are uniform across
// a block and never written while a kernel runs: read them through the
// constant address space so they arrive in scalar registers (scalar loads)
// and the interpreter's dispatch is scalar branches, not masked lanes.
template <typename Tp>
__device__ __forceinline__ Tp uniform_load(const Tp *p) {
  static_assert(sizeof(Tp) % 4 == 0, "schedule records are whole words");
  const __attribute__((address_space(4))) uint32_t *q = (const __attribute__((address_space(4))) uint32_t *)p;
  uint32_t w[sizeof(Tp) / 4];
#pragma unroll
  for (int k = 0; k < (int)(sizeof(Tp) / 4); ++k) w[k] = q[k];
  Tp v;
  __builtin_memcpy(&v, w, sizeof(Tp));
  return v;
}

// Stage a shape's twiddle table (n entries) in LDS with BS threads: each
// thread issues all its loads before its first store, so the copy costs one
// global latency rather than one per entry a thread copies.
// Stage the table by direct global-to-LDS loads instead (16 bytes per lane,
// one wavefront-wide chunk per load): no registers, and the wave goes on at
// once, its later loads overlapping these.  Each wave must wait for its
// vector memory counter (twiddles_landed) before the barrier that opens its
// first transform, and before it ends.
template <int BS, int n, typename R>
__device__ __forceinline__ void stage_twiddles_async(cpx<R> *dst, const cpx<R> *src) {
  constexpr int EPL = 16 / (int)sizeof(cpx<R>), CH = 64 * EPL, NW = BS / 64;
  static_assert(BS % 64 == 0 && EPL >= 1, "whole wavefronts, 16-byte lanes");
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / 64)), lane = threadIdx.x % 64;
  for (int c = w; c * CH < n; c += NW) {
    const int i = c * CH + lane * EPL;
    if (i < n)
      __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void *)(src + i),
                                       (__attribute__((address_space(3))) void *)(dst + c * CH), 16, 0, 0);
  }
}
__device__ __forceinline__ void twiddles_landed() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

template <int BS, int n, typename R>
__device__ __forceinline__ void stage_twiddles(cpx<R> *dst, const cpx<R> *src) {
  constexpr int K = (n + BS - 1) / BS;
  cpx<R> v[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int i = threadIdx.x + BS * k;
    if (i < n) v[k] = gload(src, i);
  }
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int i = threadIdx.x + BS * k;
    if (i < n) dst[i] = v[k];
  }
}

// LDS of a row or column body: the transform buffers, the staged twiddle
// table (when it fits; else a 16-byte stub) and the reduction slots, in that order.  The
// standalone kernels declare them as static arrays; the persistent batch
// kernel (DYN) carves them from one dynamic region that every team shape it
// hosts shares, sized on the host from these functions.
template <typename real, int T, int E, int BSZ = 0, bool PAD = (E % 3 == 0), bool LANES = false>
struct BodyLds {
  using S = Shape<T, E, BSZ, PAD>;
  static constexpr int TWN = S::template tw_in_lds<real, LANES>() ? S::N : 16 / (int)sizeof(cpx<real>);
  static constexpr int BUF = S::TPB * S::template nbuf<real, LANES>() * S::L;  // row and plain column bodies
  static constexpr int RED = 2 * (S::BS / 64);
  // per-wavefront partial maxima of the fields of a compiled program's LD2s
  static constexpr int FMX = (!LANES && BSZ == 0 && row_compiled_shapes(T, E, PAD) &&
                              S::KR * T >= kBlockMaximaCols)
                                 ? 2 * kRowShapeMaxLd2 * (S::BS / 64)
                                 : 0;
  static constexpr int bytes() {
    return (BUF + TWN) * (int)sizeof(cpx<real>) + (RED + FMX) * (int)sizeof(float);
  }
};

// One entry of a batched launch: the tile's argument record and the
// program (row pass) or task (column pass) its blocks run.
struct BatchItem {
  int32_t tile;   // index into the launch's argument table
  int32_t index;  // program or task index in that tile's schedule
};

// Row pass body: TPB teams per block, one row each (block blk of the
// pass), all running program progs[prog].
// LANES: run the transforms in the permuted layout (only for a shape whose
// lanes_ok() holds).
template <typename real, int T, int E, bool DYN = false, int BSZ = 0, bool PAD = (E % 3 == 0), bool LANES = false>
__device__ __forceinline__ void row_body(const RowArgs<real> &a, int prog, int blk, const RowProg *progs0) {
  using S = Shape<T, E, BSZ, PAD>;
  constexpr int N = S::N, L = S::L, NB = S::template nbuf<real, LANES>();
  constexpr bool TWL = S::template tw_in_lds<real, LANES>();
  static_assert(!LANES || S::template lanes_ok<real>(), "no permuted-layout form for this shape");
  // A single grid passes its program table as a kernel argument, so the
  // program record loads alongside the argument record, not after it (the
  // empty asm keeps that path a branch of its own).
  RowProg pg;
  if (progs0) {
    asm volatile("");
    pg = uniform_load(progs0 + prog);
  } else {
    pg = uniform_load(a.progs + prog);
  }
  using LD = BodyLds<real, T, E, BSZ, PAD, LANES>;
  cpx<real> *smem, *twl;
  float *red;
  if constexpr (DYN) {
    extern __shared__ __attribute__((aligned(16))) char zk_dyn_lds[];
    smem = reinterpret_cast<cpx<real> *>(zk_dyn_lds);
    twl = smem + LD::BUF;
    red = reinterpret_cast<float *>(twl + LD::TWN);
  } else {
    __shared__ cpx<real> s_smem[LD::BUF];
    __shared__ __attribute__((aligned(16))) cpx<real> s_twl[LD::TWN];
    __shared__ float s_red[LD::RED + LD::FMX];
    smem = s_smem;
    twl = s_twl;
    red = s_red;
  }
  float *fmx = red + LD::RED;  // LD::FMX floats (compiled programs only)
  const int team = threadIdx.x / T;
  const int t = threadIdx.x % T;
  // rows y and y+1 share 128-byte lines of the tiled fields
  const int row = (S::TPB == 1 ? xcd_unit(blk, a.rows, 2) : blk) * S::TPB + team;
  // A 1D grid has one row: the block's other teams run the transforms on
  // zeros (they share its barriers) and touch no field.
  const bool in_row = row < a.rows;
  cpx<real> *b0 = smem + team * NB * L;
  cpx<real> *b1 = b0 + (NB - 1) * L;
  // the permuted forms read the natural table, the others this shape's
  // pass-ordered table
  const cpx<real> *tw = a.tw + (LANES ? kTwNatural : tw_slot(E)) * N;
  if constexpr (TWL) {
    stage_twiddles_async<S::BS, LANES ? N : N - E>(twl, tw);
    tw = twl;
  }
  // No barrier here: every pass-ordered transform form of a team spanning
  // wavefronts opens with one before its first twiddle read, which publishes
  // the staged table once each wave has waited for its share (settle_tw,
  // before the first transform).  The permuted forms, and teams inside one
  // wavefront (whose transforms order their LDS within the wavefront), need
  // not open with one, so there settle_tw publishes the table with a barrier
  // of its own.
  bool tw_pending = TWL;
  auto settle_tw = [&]() {
    if (tw_pending) {
      twiddles_landed();
      if constexpr (LANES || T <= 64) __syncthreads();
      tw_pending = false;
    }
  };

  // Register sets: u = z[].x, v = z[].y (the FFT buffer), then A, o0, o1, o2.
  cpx<real> z[E];
  real R[kRowRegs - 2][E];
#pragma unroll
  for (int e = 0; e < E; ++e) z[e] = {(real)0, (real)0};
#pragma unroll
  for (int s = 0; s < kRowRegs - 2; ++s)
#pragma unroll
    for (int e = 0; e < E; ++e) R[s][e] = (real)0;
  auto reg = [&](auto Sx, int e) -> real & {
    constexpr int s = decltype(Sx)::value;
    if constexpr (s == RS_U) return z[e].x;
    else if constexpr (s == RS_V) return z[e].y;
    else return R[s - 2][e];
  };

  // The operations, shared by the interpreter and the compiled shapes.
  // maxima(op, ma, mb): the two fields' maxima over all columns
  auto do_ld2 = [&](const RowOp &op, auto &&maxima) {
    const cpx<real> *Fa = a.mix + (long long)op.fa * a.mix_stride;
    const bool has_b = op.fb >= 0;
    const cpx<real> *Fb = a.mix + (long long)(has_b ? op.fb : op.fa) * a.mix_stride;
    const bool dxa = op.fla & FL_DX, dxb = op.flb & FL_DX;
    // The two real fields share one complex transform; each is scaled by
    // a power of two from its field maximum (published by the lifts that
    // wrote it) so that neither drowns in the rounding of the other, and
    // unscaled exactly afterwards.
    // Data loads first; the field maxima (one per column, published by
    // the lifts) are reduced over all columns by each wavefront on its
    // own, so no block barrier sits between the loads and their use.
    // Padded passes up to 512-thread teams load the half spectra in the
    // layout of the transposed transform's first butterflies (element
    // p = j + NB r of butterfly j = t + T it); its result arrives in z[]
    // as element t + T e without an LDS readout.  (1024-thread teams, and
    // base lengths, whose last pass keeps only half the team busy,
    // measured faster with team_fft from the t + T e layout.)  The
    // permuted form loads element t + T e and leaves in z[s] the point
    // s + E bitrev(t / 64) + E (T / 64) bitrev6(t % 64) of the row.
    auto ld2 = [&](auto xp_c, auto lanes_c) {
      constexpr bool XP = decltype(xp_c)::value, PERMUTED = decltype(lanes_c)::value;
      using HL = HbmLayout<N, E, XP>;
      cpx<real> xa[HL::IT][HL::R], xb[HL::IT][HL::R];
      auto elem = [&](int it, int r) { return HL::elem(t, it, r); };
      auto live = [&](int it) { return HL::live(t, it); };
#pragma unroll
      for (int it = 0; it < HL::IT; ++it)
#pragma unroll
        for (int r = 0; r < HL::R; ++r) {
          const int p = elem(it, r);
          const bool pos = p < S::KR * T, neg = p > S::NEG0 * T;  // kept band, upper half by symmetry
          xa[it][r] = {(real)0, (real)0};
          xb[it][r] = {(real)0, (real)0};
          if (in_row && live(it) && (pos || neg)) {
            const int idx = mix_index<real>(pos ? p : N - p, row, a.rows);
            xa[it][r] = gload(Fa, idx);
            if (has_b) xb[it][r] = gload(Fb, idx);
          }
        }
      float ma = 0.f, mb = 0.f;
      maxima(op, ma, mb);
      const float2 pa = pow2_scale(ma);
      const float2 pb = has_b ? pow2_scale(mb) : make_float2(1.f, 1.f);
      const real sa = (real)pa.x, sb = (real)pb.x;
#pragma unroll
      for (int it = 0; it < HL::IT; ++it)
#pragma unroll
        for (int r = 0; r < HL::R; ++r) {
          const int p = elem(it, r);
          const bool pos = p < S::KR * T, neg = p > S::NEG0 * T;
          cpx<real> za = xa[it][r], zbr = xb[it][r];
          if (pos || neg) {
            const real kxv = (real)(a.kx_scale * (pos ? p : N - p));
            if (dxa) za = {-kxv * za.y, kxv * za.x};
            if (dxb) zbr = {-kxv * zbr.y, kxv * zbr.x};
            if (neg) {
              za.y = -za.y;
              zbr.y = -zbr.y;
            }
          }
          xa[it][r] = {za.x * sa - zbr.y * sb, za.y * sa + zbr.x * sb};
        }
      settle_tw();
      if constexpr (PERMUTED) {
#pragma unroll
        for (int e = 0; e < E; ++e) z[e] = xa[0][e];
        perm_ifft<real, T, E, +1>(z, b0, b1, tw, t);
      } else {
        fft_in<real, N, E, NB, +1, XP>(xa, z, b0, b1, tw, t);
      }
      const real ia = (real)pa.y, ib = (real)pb.y;
#pragma unroll
      for (int e = 0; e < E; ++e) z[e] = {z[e].x * ia, z[e].y * ib};
    };
    if constexpr (LANES) ld2(std::false_type{}, std::true_type{});
    else ld2(std::integral_constant<bool, T <= 512 && S::PADDED>{}, std::false_type{});
  };
  constexpr int NC = S::KR * T;  // nx / 2 columns: the length of a field's column maxima
  // Each wavefront reduces every column maximum of the two fields on its own
  // (no barrier between the loads and their use).
  auto wave_maxima = [&](const RowOp &op, float &ma, float &mb) {
    const float *ca = a.colmax + (long long)op.fa * NC;
    const float *cb = a.colmax + (long long)(op.fb >= 0 ? op.fb : op.fa) * NC;
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int c = lane; c < NC; c += 64) {
      ma = fmaxf(ma, gload1(ca, c));
      mb = fmaxf(mb, gload1(cb, c));
    }
    ma = wave_max(ma);
    mb = wave_max(mb);
  };
  // LDP and STP act on caller fields, whose rows have the base length only.
  auto do_ldp = [&](const RowOp &op) {
    if constexpr (!S::PADDED) {
      const double *pa = op.fa == 0 ? a.pin0 : (op.fa == 1 ? a.pin1 : a.pin2);
      const double *pb = op.fb == 0 ? a.pin0 : (op.fb == 1 ? a.pin1 : a.pin2);
      const long long off = (long long)row * a.nx;
#pragma unroll
      for (int e = 0; e < E; ++e) {
        z[e].x = in_row ? (real)gload1(pa, off + t + T * e) : (real)0;
        z[e].y = in_row && op.fb >= 0 ? (real)gload1(pb, off + t + T * e) : (real)0;
      }
    }
  };
  auto do_zero = [&]() {  // clears all three outputs
#pragma unroll
    for (int e = 0; e < E; ++e) R[RS_O0 - 2][e] = R[RS_O1 - 2][e] = R[RS_O2 - 2][e] = (real)0;
  };
  auto do_bern = [&](const RowOp &op) {
    const real eps = (real)op.coef;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const real Sv = (real)1 + eps * eps * R[RS_O0 - 2][e];
      const real W = (z[e].x + eps * R[RS_O1 - 2][e]) / Sv;
      R[RS_O0 - 2][e] = eps * ((real)-0.5 * R[RS_O2 - 2][e] + (real)0.5 * Sv * W * W);
    }
  };
  // forward transform of (u, v) once they hold the op's sources; split and store
  auto do_st2 = [&](const RowOp &op) {
    float mx = 0.f, my = 0.f;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      mx = fmaxf(mx, fabsf((float)z[e].x));
      my = fmaxf(my, fabsf((float)z[e].y));
    }
    const float2 mxy = team_max2<T>(mx, my, red);
    const float2 px = pow2_scale(mxy.x);
    const float2 py = pow2_scale(mxy.y);
    const real sx = (real)px.x, sy = (real)py.x;
#pragma unroll
    for (int e = 0; e < E; ++e) z[e] = {z[e].x * sx, z[e].y * sy};
    settle_tw();
    const cpx<real> *res;
    // (team_max2's barriers follow every earlier read of the buffers)
    if constexpr (LANES) res = perm_fft<real, T, E, -1, false>(z, b0, b1, tw, t);
    else res = team_fft<real, N, E, NB, -1>(z, b0, b1, tw, t);
    cpx<real> *Fa = a.mix + (long long)op.fa * a.mix_stride;
    cpx<real> *Fb = a.mix + (long long)(op.fb >= 0 ? op.fb : 0) * a.mix_stride;
    const real hx = (real)0.5 * (real)px.y, hy = (real)0.5 * (real)py.y;
#pragma unroll
    for (int q = 0; q < S::KR; ++q) {
      const int k = t + T * q;
      const cpx<real> zk = res[lpad(k)];
      const cpx<real> zm = res[lpad(k == 0 ? 0 : N - k)];
      const int idx = mix_index<real>(k, row, a.rows);
      if (in_row) gstore(Fa, idx, cpx<real>{hx * (zk.x + zm.x), hx * (zk.y - zm.y)});
      if (in_row && op.fb >= 0) gstore(Fb, idx, cpx<real>{hy * (zk.y + zm.y), -hy * (zk.x - zm.x)});
    }
  };
  auto do_stp = [&](const RowOp &op, auto X) {
    if constexpr (!S::PADDED) {
      double *po = op.fa == 0 ? a.pout0 : a.pout1;
      const long long off = ((long long)(op.fb > 0 ? op.fb : 0) * a.rows + row) * a.nx;
#pragma unroll
      for (int e = 0; e < E; ++e)
        if (in_row) gstore1(po, off + t + T * e, (double)reg(X, e));
    }
  };

  // A program of a compiled shape runs as straight-line code: its register
  // sets are fixed at compile time, so no interpreter state merges between
  // operations (and no operation dispatch remains); only the field ids, flags
  // and coefficients come from the op records.
  if constexpr (row_compiled_shapes(T, E, S::PADDED) && !DYN && !LANES && BSZ == 0) {
    if (pg.shape1 > 0) {
      static_for<0, kRowShapes>([&](auto shc) {
        constexpr int SH = decltype(shc)::value;
        if (pg.shape1 == SH + 1) {
          // Rows of at least 2048 points (1024 column maxima per field): the
          // column maxima of every LD2's fields are reduced once per block up
          // front (each wavefront a share of the columns, one barrier)
          // instead of in full by every wavefront at each LD2 (a quarter
          // faster row pass at 2048 points; no gain at 1024, a loss at 512).
          // Shorter rows keep the per-wavefront reductions.
          constexpr bool BLOCK_MAXIMA = NC >= kBlockMaximaCols;
          constexpr int NW = S::BS / 64;
          const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
          static_for<0, kRowShapeLen[SH]>([&](auto ic) {
            constexpr int I = decltype(ic)::value;
            if constexpr (BLOCK_MAXIMA && (kRowShapeOps[SH][I] & 255) == OP_LD2) {
              constexpr int J = row_shape_ld2_ordinal(SH, I);
              const RowOp op = uniform_load(a.ops + pg.op0 + I);
              const float *ca = a.colmax + (long long)op.fa * NC;
              const float *cb = a.colmax + (long long)(op.fb >= 0 ? op.fb : op.fa) * NC;
              float ma = 0.f, mb = 0.f;
#pragma unroll
              for (int c = wv * 64 + lane; c < NC; c += NW * 64) {
                ma = fmaxf(ma, gload1(ca, c));
                mb = fmaxf(mb, gload1(cb, c));
              }
              ma = wave_max(ma);
              mb = wave_max(mb);
              if (lane == 0) {
                fmx[(2 * J) * NW + wv] = ma;
                fmx[(2 * J + 1) * NW + wv] = mb;
              }
            }
          });
          if constexpr (BLOCK_MAXIMA) __syncthreads();
          static_for<0, kRowShapeLen[SH]>([&](auto ic) {
            constexpr int I = decltype(ic)::value;
            constexpr uint32_t w = kRowShapeOps[SH][I];
            constexpr int code = w & 255, A = (w >> 8) & 255, B = (w >> 16) & 255, C = (int)(w >> 24);
            using IA = std::integral_constant<int, A>;
            using IB = std::integral_constant<int, B>;
            using IC = std::integral_constant<int, C>;
            const RowOp op = uniform_load(a.ops + pg.op0 + I);
            if constexpr (code == OP_LD2 && BLOCK_MAXIMA) {
              constexpr int J = row_shape_ld2_ordinal(SH, I);
              do_ld2(op, [&](const RowOp &, float &ma, float &mb) {
#pragma unroll
                for (int k = 0; k < NW; ++k) {
                  ma = fmaxf(ma, fmx[(2 * J) * NW + k]);
                  mb = fmaxf(mb, fmx[(2 * J + 1) * NW + k]);
                }
              });
            } else if constexpr (code == OP_LD2) {
              do_ld2(op, wave_maxima);
            } else if constexpr (code == OP_MOV) {
#pragma unroll
              for (int e = 0; e < E; ++e) R[RS_A - 2][e] = reg(IB{}, e);
            } else if constexpr (code == OP_MAC) {
              const real c = (real)op.coef;
#pragma unroll
              for (int e = 0; e < E; ++e) {
                const real pr = reg(IB{}, e) * reg(IC{}, e);
                reg(IA{}, e) += c * pr;
              }
            } else if constexpr (code == OP_ZERO) {
              do_zero();
            } else if constexpr (code == OP_BERN) {
              do_bern(op);
            } else if constexpr (code == OP_ST2) {
              if constexpr (A != RS_U) {
#pragma unroll
                for (int e = 0; e < E; ++e) z[e].x = reg(IA{}, e);
              }
              if constexpr (B == RS_NONE) {
#pragma unroll
                for (int e = 0; e < E; ++e) z[e].y = (real)0;
              } else if constexpr (B != RS_V) {
#pragma unroll
                for (int e = 0; e < E; ++e) z[e].y = reg(IB{}, e);
              }
              do_st2(op);
            }
            // each operation's instructions stay together, as in the
            // interpreter (measured: the same registers and speed without)
            __builtin_amdgcn_sched_barrier(0);
          });
        }
      });
      settle_tw();  // no load into LDS may outlive the block
      return;
    }
  }

  for (int i = 0; i < pg.nop; ++i) {
    const RowOp op = uniform_load(a.ops + pg.op0 + i);
    switch (op.code) {
      case OP_LD2:
        do_ld2(op, wave_maxima);
        break;
      case OP_LDP:
        do_ldp(op);
        break;
      // MOV, MAC and ZERO write their targets without a branch on the target
      // register: a switch per target would make the compiler copy every
      // register set at each merge of the interpreter loop.
      case OP_MOV: {  // A <- u, v or A
        real m[E];
        with_in(op.b, [&](auto Sx) {
#pragma unroll
          for (int e = 0; e < E; ++e) m[e] = reg(Sx, e);
        });
#pragma unroll
        for (int e = 0; e < E; ++e) R[RS_A - 2][e] = m[e];
        break;
      }
      case OP_MAC: {  // o[a] += coef * x * y, as weighted adds to all three outputs
        const real c = (real)op.coef;
        const real w0 = op.a == RS_O0 ? c : (real)0, w1 = op.a == RS_O1 ? c : (real)0,
                   w2 = op.a == RS_O2 ? c : (real)0;
        real pr[E];
        with_in(op.b, [&](auto X) {
          with_in(op.c, [&](auto Y) {
#pragma unroll
            for (int e = 0; e < E; ++e) pr[e] = reg(X, e) * reg(Y, e);
          });
        });
#pragma unroll
        for (int e = 0; e < E; ++e) {
          R[RS_O0 - 2][e] += w0 * pr[e];
          R[RS_O1 - 2][e] += w1 * pr[e];
          R[RS_O2 - 2][e] += w2 * pr[e];
        }
        break;
      }
      case OP_ZERO:
        do_zero();
        break;
      case OP_BERN:
        do_bern(op);
        break;
      case OP_ST2: {
        // Sources are (u, v) in place, or sets outside the FFT buffer (the
        // planner never pairs u or v with another set).
        if (op.a != RS_U) {
          with_any(op.a, [&](auto X) {
#pragma unroll
            for (int e = 0; e < E; ++e) z[e].x = reg(X, e);
          });
        }
        if (op.b == RS_NONE) {
#pragma unroll
          for (int e = 0; e < E; ++e) z[e].y = (real)0;
        } else if (op.b != RS_V) {
          with_any(op.b, [&](auto Y) {
#pragma unroll
            for (int e = 0; e < E; ++e) z[e].y = reg(Y, e);
          });
        }
        do_st2(op);
        break;
      }
      case OP_STP:
        with_any(op.a, [&](auto X) { do_stp(op, X); });
        break;
      default:
        break;
    }
  }
  settle_tw();  // no load into LDS may outlive the block
}

// ---------------------------------------------------------------------------
// Factors of the bulk velocity lift, applied at the lift stage of a column
// task (one site, after the terms are summed, so the exponentials do not
// raise the register peak of the pass).  COUPLE: prod_a exp(-(|k_a| / (kNyq_a / 2))^8).  LAYER_C / _S:
// C = cosh(k (d - y)) / cosh(k d), S = k sinh(k (d - y)) / cosh(k d) at the
// chunk's layer depth y, as exp(-k y) (1 +- exp(-2 k (d - y))) / (1 + exp(-2 k d));
// deep water: exp(-k y) and k exp(-k y); C = 1, S = 0 at k = 0.
__device__ __forceinline__ double lift_factor(uint32_t s, double kk, int col, int b, int nx, int ny, double depth,
                                           const double *layer_y) {
  double f = 1.0;
  if (s & SYM_COUPLE) {
    const int my = (b < ny / 2 || ny == 1) ? b : b - ny;  // a 1D grid's one row is ky = 0
    const double rx = 4.0 * col / nx, ry = 4.0 * (my < 0 ? -my : my) / ny;  // |k_a| / (kNyq_a / 2)
    const double rx2 = rx * rx, ry2 = ry * ry, rx4 = rx2 * rx2, ry4 = ry2 * ry2;
    f *= exp(-(rx4 * rx4) - (ry4 * ry4));
  }
  if (s & (SYM_LAYER_C | SYM_LAYER_S)) {
    const double y = layer_y[(s >> SYM_LAYER_SHIFT) & 15];
    double c = 1.0, sn = 0.0;
    if (kk > 0.0) {
      const double e1 = exp(-kk * y);
      if (depth > 0.0) {
        const double e2 = exp(-2.0 * kk * (depth - y)), den = 1.0 + exp(-2.0 * kk * depth);
        c = e1 * (1.0 + e2) / den;
        sn = kk * e1 * (1.0 - e2) / den;
      } else {
        c = e1;
        sn = kk * e1;
      }
    }
    f *= (s & SYM_LAYER_S) ? sn : c;
  }
  return f;
}

// ---------------------------------------------------------------------------
// Fourier symbols at (kx, b) of the base band, from tables computed once on
// the host in FP64: |k|, G0 = |k| tanh(|k| d) and the taper, per band element
// (same tiled layout as a base spectrum); the state filter is separable,
// A = Ax(kx) Ay(b).
template <typename real>
__device__ __forceinline__ cpx<double> symval(uint32_t s, double kk, double g0, double tp, int col, int b,
                                              double ky, const ColArgs<real> &a) {
  double f = 1.0;
  const int l = s & SYM_LMASK;
  if (l) {  // L_l = G0 |k|^(l-1) for odd l, |k|^l for even l
    f = (l & 1) ? g0 : kk;
    for (int i = 1; i < l; ++i) f *= kk;
  }
  if (s & SYM_FILT) f *= gload1(a.filt_x, col) * gload1(a.filt_y, b);
  if ((s & SYM_TAPER) && a.taper_on) f *= tp;
  if (s & SYM_IF) f *= gload1(a.ifsym, (long long)base_index(col, b, a.ny) * kIfCoefs + ((s >> SYM_IF_SHIFT) & 7));
  if (s & SYM_INVG0) f = g0 > 0.0 ? f / g0 : 0.0;
  if (s & SYM_IKY) return {0.0, f * ky};
  return {f, 0.0};
}

// Column pass body.  FT = 1: TPB teams per block (block blk of the pass),
// one kx column each, all running task tasks[task], folds one after another.
// FT = kMaxFolds (fold teams): the block's FT teams share one column; team f
// transforms fold f and sums a share of each output's terms, the parts are
// summed through LDS in team order, so a task with several folds and long
// term lists runs them side by side instead of in sequence.  Thread t owns
// base-band rows b = t + T q, q < QB (q = KR at t = 0 is the ky Nyquist row,
// kept zero).
template <int T, int FT, int BSZ = 0>
struct ColBlock {
  static constexpr int BS = FT == 1 ? (BSZ ? BSZ : (T > 256 ? T : 256)) : FT * T;  // threads per block
  static constexpr int TPB = FT == 1 ? BS / T : 1;                    // columns per block
};
template <typename real, int T, int E, bool LIFTSYM = false, int FT = 1, bool DYN = false, int BSZ = 0,
          bool PAD = (E % 3 == 0)>
__device__ __forceinline__ void col_body(const ColArgs<real> &a, int task_index, int blk, const ColTask *tasks0) {
  static_assert(BSZ == 0 || FT == 1, "a block size is set for plain column teams only");
  using S = Shape<T, E, BSZ, PAD>;
  using CB = ColBlock<T, FT, BSZ>;
  static_assert(FT == 1 || (T >= 64 && FT * T <= 1024), "fold teams: whole wavefronts, one block");
  constexpr int N = S::N, L = S::L, QB = S::QB;
  constexpr int NB = FT == 1 ? S::template nbuf<real>() : 2;
  constexpr bool TWL = FT == 1 ? S::template tw_in_lds<real>() : true;
  // (a single grid passes its task table too: see row_body)
  ColTask task;
  if (tasks0) {
    asm volatile("");
    task = uniform_load(tasks0 + task_index);
  } else {
    task = uniform_load(a.tasks + task_index);
  }
  static_assert(!DYN || FT == 1, "the persistent kernel hosts plain column teams only");
  constexpr int TWN = TWL ? N : 16 / (int)sizeof(cpx<real>);
  cpx<real> *smem, *twl;
  float *red;
  cpx<double> *xs;
  if constexpr (DYN) {
    using LD = BodyLds<real, T, E, BSZ, PAD>;
    extern __shared__ __attribute__((aligned(16))) char zk_dyn_lds[];
    smem = reinterpret_cast<cpx<real> *>(zk_dyn_lds);
    twl = smem + LD::BUF;
    red = reinterpret_cast<float *>(twl + LD::TWN);
    xs = nullptr;
  } else {
    __shared__ cpx<real> s_smem[(FT == 1 ? CB::TPB : FT) * NB * L];
    __shared__ __attribute__((aligned(16))) cpx<real> s_twl[TWN];
    __shared__ float s_red[2 * (CB::BS / 64)];
    __shared__ cpx<double> s_xs[FT == 1 ? 1 : FT * QB * T];  // fold teams: each team's part of X
    smem = s_smem;
    twl = s_twl;
    red = s_red;
    xs = s_xs;
  }
  // fold teams are whole wavefronts: the team index is wave-uniform (scalar)
  const int team = FT == 1 ? (int)(threadIdx.x / T) : __builtin_amdgcn_readfirstlane((int)(threadIdx.x / T));
  const int t = threadIdx.x % T;
  // columns of one tile share 128-byte lines; keep a tile's blocks on one XCD
  constexpr int CBMAX = MixTile<real>::CB > CBB ? MixTile<real>::CB : CBB;
  const int col_raw = FT == 1 ? xcd_unit(blk, a.nx / 2 / CB::TPB, CBMAX / CB::TPB) * CB::TPB + team
                              : xcd_unit(blk, a.nx / 2, CBMAX);
  // A grid with fewer columns than a block has teams (nx / 2 < 256 / T):
  // the spare teams run the last column's transforms alongside (they share
  // its barriers) and store nothing.
  const bool in_col = col_raw < a.nx / 2;
  const int col = in_col ? col_raw : a.nx / 2 - 1;
  cpx<real> *b0 = smem + team * NB * L;
  cpx<real> *b1 = b0 + (NB - 1) * L;
  const int ny = a.ny;
  const cpx<real> *tw = a.tw + tw_slot(E) * N;  // this shape's pass-ordered table
  if constexpr (TWL) {
    stage_twiddles_async<CB::BS, N - E>(twl, tw);
    tw = twl;
  }
  // (no barrier: the first transform's opening barrier publishes the table,
  // once each wave has waited for its share in settle_tw)
  bool tw_pending = TWL;
  auto settle_tw = [&]() {
    if (tw_pending) {
      twiddles_landed();
      if constexpr (T <= 64) __syncthreads();  // one-wavefront teams' transforms open without one
      tw_pending = false;
    }
  };

  auto my_of = [&](int q) {
    const int b = t + T * q;
    return (b < ny / 2) ? b : b - ny;
  };
  // |k| from the wavenumbers; G0 and the taper from their tables only where
  // the problem and the task have them (a task's symbols read them for every
  // band element, which at large grids is a fair share of the pass's memory
  // traffic).  Only folds carry the taper (the plan validation holds output
  // terms to that).
  const bool need_tp = a.taper_on && ((task.fwd_sym[0] | task.fwd_sym[1] | task.fwd_sym[2]) & SYM_TAPER);
  double skk[QB], sg0[QB], stp[QB];
#pragma unroll
  for (int q = 0; q < QB; ++q) {
    const long long e = base_index(col, t + T * q, ny);
    const double kx = a.kx_scale * col, ky = a.ky_scale * my_of(q);
    skk[q] = sqrt(kx * kx + ky * ky);
    sg0[q] = a.depth > 0.0 ? gload1(a.sym_g0, e) : skk[q];
    stp[q] = need_tp ? gload1(a.sym_tp, e) : 1.0;
  }
  auto sym = [&](uint32_t s, int q) -> cpx<double> {
    return symval(s, skk[q], sg0[q], stp[q], col, t + T * q, a.ky_scale * my_of(q), a);
  };

  cpx<double> X[QB];
#pragma unroll
  for (int q = 0; q < QB; ++q) X[q] = {0.0, 0.0};
  // Padded passes up to 512-thread teams run folds on the transposed
  // transform (the column is loaded in the layout of its first butterflies)
  // and keep a lift's last pass in registers (stored from there), each an
  // LDS round trip fewer; 1024-thread teams and base lengths (measured
  // faster without) and the depth-lift variant (whose registers these forms
  // would push past an occupancy step) use team_fft with LDS readouts.
  // Either way a fold's result is element t + T r in v[r]; base element q
  // sits at padded (or base) position t + T base_slot(q).
  constexpr bool XP = T <= 512 && S::PADDED && !LIFTSYM, KEEP = XP;
  using HL = HbmLayout<N, E, XP>;
  using HO = HbmLayout<N, E, true>;
  auto base_slot = [](int q) { return q < S::KR ? q : q + (S::PADDED ? E / 3 : 0); };
  auto load_col = [&](const cpx<real> *F, HbmRegs<real, N, E, XP> &x) {
#pragma unroll
    for (int it = 0; it < HL::IT; ++it)
#pragma unroll
      for (int r = 0; r < HL::R; ++r)
        x[it][r] = HL::live(t, it) ? gload(F, mix_index<real>(col, HL::elem(t, it, r), a.rows))
                                   : cpx<real>{(real)0, (real)0};
  };
  // get(r): element t + T r of the fold's transform
  auto fold_into = [&](auto get, uint32_t fsym, double fcoef) {
#pragma unroll
    for (int q = 0; q < QB; ++q) {
      const cpx<real> w = get(base_slot(q));
      const cpx<double> sv = sym(fsym, q);
      const cpx<double> x = {(double)w.x * fcoef, (double)w.y * fcoef};
      X[q].x += x.x * sv.x - x.y * sv.y;
      X[q].y += x.x * sv.y + x.y * sv.x;
    }
  };
  // transform x (HBM-side layout) and fold it: XP from registers, else
  // read from LDS as it is needed
  auto transform_fold = [&](HbmRegs<real, N, E, XP> &x, uint32_t fsym, double fcoef, bool use) {
    settle_tw();
    if constexpr (XP) {
      cpx<real> v[E];
      team_fft_t<real, N, E, NB, -1>(x, v, b0, b1, tw, t);
      if (use) fold_into([&](int r) { return v[r]; }, fsym, fcoef);
    } else {
      cpx<real> v[E];
#pragma unroll
      for (int r = 0; r < E; ++r) v[r] = x[0][r];
      const cpx<real> *res = team_fft<real, N, E, NB, -1>(v, b0, b1, tw, t);
      if (use) fold_into([&](int r) { return res[lpad(t + T * r)]; }, fsym, fcoef);
    }
  };
  if constexpr (FT == 1) {
    // Folds: the next field's column is loaded while the current one is
    // transformed (folds are consecutive from slot 0).
    cpx<real> xn[HL::IT][HL::R];
    auto load_fold = [&](int f) { load_col(a.mix + (long long)task.fwd[f] * a.mix_stride, xn); };
    if (task.fwd[0] >= 0) load_fold(0);
    for (int f = 0; f < kMaxFolds; ++f) {
      if (task.fwd[f] < 0) break;
      cpx<real> x[HL::IT][HL::R];
#pragma unroll
      for (int it = 0; it < HL::IT; ++it)
#pragma unroll
        for (int r = 0; r < HL::R; ++r) x[it][r] = xn[it][r];
      if (f + 1 < kMaxFolds && task.fwd[f + 1] >= 0) load_fold(f + 1);
      transform_fold(x, task.fwd_sym[f], task.fwd_coef[f], true);
    }
  } else if (task.fwd[0] >= 0) {
    // Team f folds field f (a team without one transforms zeros); the parts
    // are summed in fold order, X = ((X_0 + X_1) + X_2).
    int fid = -1;
    uint32_t fsym = 0;
    double fcoef = 0.0;
#pragma unroll
    for (int f = 0; f < FT; ++f)
      if (team == f) {
        fid = task.fwd[f];
        fsym = task.fwd_sym[f];
        fcoef = task.fwd_coef[f];
      }
    cpx<real> x[HL::IT][HL::R];
#pragma unroll
    for (int it = 0; it < HL::IT; ++it)
#pragma unroll
      for (int r = 0; r < HL::R; ++r) x[it][r] = {(real)0, (real)0};
    if (fid >= 0) load_col(a.mix + (long long)fid * a.mix_stride, x);
    transform_fold(x, fsym, fcoef, fid >= 0);
#pragma unroll
    for (int q = 0; q < QB; ++q) xs[(team * QB + q) * T + t] = X[q];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < QB; ++q) {
      X[q] = xs[q * T + t];
#pragma unroll
      for (int f = 1; f < FT; ++f) {
        const cpx<double> y = xs[(f * QB + q) * T + t];
        X[q].x += y.x;
        X[q].y += y.y;
      }
    }
  }
  if (t == 0) X[S::KR] = {0.0, 0.0};  // ky Nyquist row

  // Outputs, one after another.  FT = 1: the team sums every term.  Fold
  // teams: team f sums terms f, f + FT, ... (a third of the chain of
  // base-spectrum loads each), the parts are summed through LDS in team
  // order, and every team then holds the combination; team 0 stores it.
  for (int o = 0; o < task.no; ++o) {
    const ColOut out = uniform_load(a.outs + task.o0 + o);
    constexpr int step = FT;
    const int first = FT == 1 ? 0 : team;
    cpx<double> acc[QB];
#pragma unroll
    for (int q = 0; q < QB; ++q) acc[q] = {0.0, 0.0};
    // Base-spectrum terms: the next term's spectrum is loaded while the
    // current one is accumulated (one global latency per term instead of two).
    cpx<double> nxt[QB];
    ColTerm ntm = first < out.nt ? uniform_load(a.terms + out.t0 + first) : ColTerm{};
    auto fetch = [&](const ColTerm &tm2) {
      if (tm2.src >= 0) {
        const cpx<double> *B = a.base + (long long)tm2.src * a.base_stride;
#pragma unroll
        for (int q = 0; q < QB; ++q) nxt[q] = gload(B, base_index(col, t + T * q, ny));
      }
    };
    fetch(ntm);
    for (int i = first; i < out.nt; i += step) {
      const ColTerm tm = ntm;
      cpx<double> cur[QB];
#pragma unroll
      for (int q = 0; q < QB; ++q) cur[q] = nxt[q];
      if (i + step < out.nt) {
        ntm = uniform_load(a.terms + out.t0 + i + step);
        fetch(ntm);
      }
      if (tm.src >= 0) {
#pragma unroll
        for (int q = 0; q < QB; ++q) {
          const cpx<double> s0 = cur[q];
          cpx<double> sv = sym(tm.sym, q);
          sv = {sv.x * tm.coef, sv.y * tm.coef};
          acc[q].x += s0.x * sv.x - s0.y * sv.y;
          acc[q].y += s0.x * sv.y + s0.y * sv.x;
        }
      } else {
#pragma unroll
        for (int q = 0; q < QB; ++q) {
          cpx<double> sv = sym(tm.sym, q);
          sv = {sv.x * tm.coef, sv.y * tm.coef};
          acc[q].x += X[q].x * sv.x - X[q].y * sv.y;
          acc[q].y += X[q].x * sv.y + X[q].y * sv.x;
        }
      }
    }
    if constexpr (FT > 1) {
      __syncthreads();  // xs: readers of the previous exchange are done
#pragma unroll
      for (int q = 0; q < QB; ++q) xs[(team * QB + q) * T + t] = acc[q];
      __syncthreads();
#pragma unroll
      for (int q = 0; q < QB; ++q) {
        acc[q] = xs[q * T + t];
#pragma unroll
        for (int f = 1; f < FT; ++f) {
          const cpx<double> y = xs[(f * QB + q) * T + t];
          acc[q].x += y.x;
          acc[q].y += y.y;
        }
      }
    }
    if (t == 0) acc[S::KR] = {0.0, 0.0};
    const bool writer = (FT == 1 || team == 0) && in_col;  // fold teams: team 0 writes
    if (out.dst_base >= 0 && writer) {
      cpx<double> *B = a.base + (long long)out.dst_base * a.base_stride;
#pragma unroll
      for (int q = 0; q < QB; ++q) gstore(B, base_index(col, t + T * q, ny), acc[q]);
    }
    if (out.dst_mixed >= 0) {
      const double lc = out.lift_coef;
      cpx<real> z[E];
#pragma unroll
      for (int r = 0; r < E; ++r) z[r] = {(real)0, (real)0};
#pragma unroll
      for (int q = 0; q < QB; ++q) {
        const int r = q < S::KR ? q : q + (S::PADDED ? E / 3 : 0);
        double f = lc;
        if constexpr (LIFTSYM)
          if (out.lift_sym) f *= lift_factor(out.lift_sym, skk[q], col, t + T * q, a.nx, ny, a.depth, a.layer_y);
        z[r] = {(real)(acc[q].x * f), (real)(acc[q].y * f)};
      }
      float m = 0.f;
      cpx<real> *F = a.mix + (long long)out.dst_mixed * a.mix_stride;
      auto put = [&](int e, const cpx<real> &w) {  // element e of the lifted column (writers only)
        gstore(F, mix_index<real>(col, e, a.rows), w);
        m = fmaxf(m, fmaxf(fabsf((float)w.x), fabsf((float)w.y)));
      };
      // fold teams: every team transformed the same combination, team 0 writes
      settle_tw();
      if constexpr (KEEP) {
        cpx<real> o[HO::IT][HO::R];
        team_fft_keep<real, N, E, NB, +1>(z, b0, b1, tw, t, o);
        if (writer)
#pragma unroll
          for (int it = 0; it < HO::IT; ++it)
            if (HO::live(t, it))
#pragma unroll
              for (int r = 0; r < HO::R; ++r) put(HO::elem(t, it, r), o[it][r]);
      } else {
        const cpx<real> *res = team_fft<real, N, E, NB, +1>(z, b0, b1, tw, t);
        if (writer)
#pragma unroll
          for (int r = 0; r < E; ++r) put(t + T * r, res[lpad(t + T * r)]);
      }
      m = team_max<T>(m, red);
      if (t == 0 && writer) gstore1(a.colmax, (long long)out.dst_mixed * (a.nx / 2) + col, m);
    }
  }
  settle_tw();  // no load into LDS may outlive the block
}

// Caller fields of a single-grid call; they replace the argument record's
// field pointers when use != 0 (batches keep theirs in the record).
struct PhysArgs {
  const double *in0, *in1, *in2;
  double *out0, *out1;
  int use;
};

// The row and column kernels: blockIdx.y selects an item (argument record
// and program or task); every item of one launch shares the team shape
// (T, E), so blockIdx.x spans the same rows or columns for each.  A single
// grid is the batch of one tile; it passes no item table (items = null) but
// its record index and first program or task (tile0, first0) and its program
// or task table (sched0), which arrive preloaded in registers, so a block's
// first loads wait neither on an item nor on the argument record.
__device__ __forceinline__ BatchItem item_of(const BatchItem *items, int tile0, int first0) {
  return items ? items[blockIdx.y] : BatchItem{tile0, first0 + (int)blockIdx.y};
}
template <typename real, int T, int E, bool PAD = (E % 3 == 0), bool LANES = false>
__global__ __launch_bounds__(T > 256 ? T : 256) void row_kernel_batch(const RowArgs<real> *__restrict__ args,
                                                        const BatchItem *__restrict__ items, int tile0, int first0,
                                                        const void *sched0, PhysArgs ph) {
  const BatchItem it = item_of(items, tile0, first0);
  RowArgs<real> a = args[it.tile];
  if (ph.use) {
    a.pin0 = ph.in0;
    a.pin1 = ph.in1;
    a.pin2 = ph.in2;
    a.pout0 = ph.out0;
    a.pout1 = ph.out1;
  }
  row_body<real, T, E, false, 0, PAD, LANES>(a, it.index, blockIdx.x, static_cast<const RowProg *>(sched0));
}
// LIFTSYM: the variant that applies ColOut.lift_sym (the bulk velocity
// lift's column launches); the plain passes never carry its exponentials.
template <typename real, int T, int E, bool LIFTSYM = false, bool PAD = (E % 3 == 0)>
__global__ __launch_bounds__(T > 256 ? T : 256) void col_kernel_batch(const ColArgs<real> *__restrict__ args,
                                                        const BatchItem *__restrict__ items, int tile0, int first0,
                                                        const void *sched0, PhysArgs) {
  const BatchItem it = item_of(items, tile0, first0);
  const ColArgs<real> a = args[it.tile];
  col_body<real, T, E, LIFTSYM, 1, false, 0, PAD>(a, it.index, blockIdx.x, static_cast<const ColTask *>(sched0));
}
// Fold teams: kMaxFolds teams of T threads per block, one column per block
// (tasks whose folds and terms run side by side).
template <typename real, int T, int E>
__global__ __launch_bounds__(kMaxFolds * T) void col_kernel_folds(const ColArgs<real> *__restrict__ args,
                                                             const BatchItem *__restrict__ items, int tile0,
                                                             int first0, const void *sched0, PhysArgs) {
  const BatchItem it = item_of(items, tile0, first0);
  const ColArgs<real> a = args[it.tile];
  col_body<real, T, E, false, kMaxFolds>(a, it.index, blockIdx.x, static_cast<const ColTask *>(sched0));
}

// Column pass of a 1D grid (ny = 1): a kx column holds the single ky = 0
// element, so a fold is that element (a one-point transform, no truncation
// in y and no ky Nyquist row) and a lift writes it back; one thread per
// column, the same task records as col_body.
template <typename real, bool LIFTSYM>
__device__ __forceinline__ void col_body_1d(const ColArgs<real> &a, int task_index, int col) {
  const ColTask task = uniform_load(a.tasks + task_index);
  if (col >= a.nx / 2) return;  // no barriers in this body
  const long long e = base_index(col, 0, 1);
  const double kk = a.kx_scale * col;  // ky = 0
  const bool need_tp = a.taper_on && ((task.fwd_sym[0] | task.fwd_sym[1] | task.fwd_sym[2]) & SYM_TAPER);
  const double g0 = a.depth > 0.0 ? gload1(a.sym_g0, e) : kk, tp = need_tp ? gload1(a.sym_tp, e) : 1.0;
  auto sym = [&](uint32_t s) { return symval(s, kk, g0, tp, col, 0, 0.0, a); };
  auto cmac = [](cpx<double> &acc, cpx<double> x, cpx<double> sv) {
    acc.x += x.x * sv.x - x.y * sv.y;
    acc.y += x.x * sv.y + x.y * sv.x;
  };
  cpx<double> X = {0.0, 0.0};
  for (int f = 0; f < kMaxFolds; ++f) {
    if (task.fwd[f] < 0) break;
    const cpx<real> w = gload(a.mix + (long long)task.fwd[f] * a.mix_stride, mix_index<real>(col, 0, a.rows));
    cmac(X, cpx<double>{(double)w.x * task.fwd_coef[f], (double)w.y * task.fwd_coef[f]}, sym(task.fwd_sym[f]));
  }
  for (int o = 0; o < task.no; ++o) {
    const ColOut out = uniform_load(a.outs + task.o0 + o);
    cpx<double> acc = {0.0, 0.0};
    for (int i = 0; i < out.nt; ++i) {
      const ColTerm tm = uniform_load(a.terms + out.t0 + i);
      const cpx<double> src =
          tm.src >= 0 ? gload(a.base + (long long)tm.src * a.base_stride, base_index(col, 0, 1)) : X;
      cpx<double> sv = sym(tm.sym);
      cmac(acc, src, cpx<double>{sv.x * tm.coef, sv.y * tm.coef});
    }
    if (out.dst_base >= 0) gstore(a.base + (long long)out.dst_base * a.base_stride, base_index(col, 0, 1), acc);
    if (out.dst_mixed >= 0) {
      double f = out.lift_coef;
      if constexpr (LIFTSYM)
        if (out.lift_sym) f *= lift_factor(out.lift_sym, kk, col, 0, a.nx, 1, a.depth, a.layer_y);
      const cpx<real> w = {(real)(acc.x * f), (real)(acc.y * f)};
      gstore(a.mix + (long long)out.dst_mixed * a.mix_stride, mix_index<real>(col, 0, a.rows), w);
      gstore1(a.colmax, (long long)out.dst_mixed * (a.nx / 2) + col, fmaxf(fabsf((float)w.x), fabsf((float)w.y)));
    }
  }
}
template <typename real, bool LIFTSYM>
__global__ __launch_bounds__(256) void col_kernel_1d(const ColArgs<real> *__restrict__ args, int rec, int first0) {
  col_body_1d<real, LIFTSYM>(args[rec], first0 + (int)blockIdx.y, (int)(blockIdx.x * blockDim.x + threadIdx.x));
}
// Column pass of a 1D grid: grid.x covers the nx/2 columns with 256 threads
// per block, grid.y the launch's tasks; args[rec] is the pass's record.
template <typename real>
hipError_t launch_col_1d(bool liftsym, dim3 grid, hipStream_t s, const ColArgs<real> *args, int rec, int first0) {
  if (liftsym)
    hipLaunchKernelGGL((col_kernel_1d<real, true>), grid, dim3(256), 0, s, args, rec, first0);
  else
    hipLaunchKernelGGL((col_kernel_1d<real, false>), grid, dim3(256), 0, s, args, rec, first0);
  return hipGetLastError();
}

// Team shapes (T, E) compiled for the batched kernels.  Power-of-two axes
// (n = 2^k in [4, 2048]): T in {2, 4, 8, 16} with E in {2, 3, 4, 6}, T in
// {32, 64, 128, 256} threads with E in {2, 3, 4, 6, 8, 12}, and T = 512 (E in
// {2, 3, 4, 6}) and 1024 (E in {2, 3})
// as blocks of their own, so each length has two to four candidates for its
// padded (3n/2, E in {3, 6, 12}) and base (n, E in {2, 4, 8}) transforms;
// the autotuner picks among them.  Axes with a factor 3 (n = 3 2^k in [12,
// 1536]): the padded transform of 9 2^(k-1) points with E = 9 and the base
// transform with E = 6, T in {2, ..., 256}; with a factor 5 (n = 5 2^k in
// [20, 1280]): padded E = 15 and base E = 10, T in {2, ..., 128}.  `pad` tells a base transform
// with E = 6 from a padded one.  A block has max(256, T) threads.  These
// return the kernel for (T, E, pad), or nullptr if that shape is not built.
template <typename real>
const void *batch_row_kernel(int T, int E, bool pad);
template <typename real>
const void *batch_col_kernel(int T, int E, bool pad);
template <>
const void *batch_row_kernel<double>(int T, int E, bool pad);
template <>
const void *batch_row_kernel<float>(int T, int E, bool pad);
template <>
const void *batch_col_kernel<double>(int T, int E, bool pad);
template <>
const void *batch_col_kernel<float>(int T, int E, bool pad);
// The default first-pass radix of an axis of n base points: the smallest
// compiled one (n = 2^k: 3 padded, 2 base; n = 3 2^k: 9 padded, 6 base;
// n = 5 2^k: 15 padded, 10 base).
inline int default_radix(int n, bool pad) {
  return n % 5 == 0 ? (pad ? 15 : 10) : (n % 3 ? (pad ? 3 : 2) : (pad ? 9 : 6));
}
// The compiled first-pass radices of that axis's padded or base transform
// (the autotuner's candidates): writes up to three into e, returns the count.
inline int radix_candidates(int n, bool pad, int *e) {
  if (n % 3 == 0 || n % 5 == 0) {
    e[0] = default_radix(n, pad);
    return 1;
  }
  e[0] = pad ? 3 : 2;
  e[1] = pad ? 6 : 4;
  e[2] = pad ? 12 : 8;
  return 3;
}
// Axis lengths the kernels are built for: 2^k in [4, 2048], 3 2^k in [12,
// 1536] and 5 2^k in [20, 1280].
inline bool axis_len_ok(int n) {
  const int f = n % 3 == 0 ? 3 : (n % 5 == 0 ? 5 : 1);
  const int m = n / f;
  if (n % f || m <= 0 || (m & (m - 1))) return false;
  return f == 1 ? (n >= 4 && n <= 2048) : (f == 3 ? (n >= 12 && n <= 1536) : (n >= 20 && n <= 1280));
}
// Launch the kernel of shape (T, E, pad) (hipErrorInvalidValue if not built).
template <typename real>
hipError_t launch_batch_row(int T, int E, bool pad, dim3 grid, hipStream_t s, const RowArgs<real> *args,
                            const BatchItem *items, int tile0, int first0, const void *sched0, PhysArgs ph);
// The padded row kernels in the permuted-layout form (ZK_ROW_FFT_LANES),
// built for every padded row shape with row_lanes_ok: the kernel, or nullptr;
// the launch, or hipErrorInvalidValue.
template <typename real>
const void *lanes_row_kernel(int T, int E);
template <>
const void *lanes_row_kernel<double>(int T, int E);
template <>
const void *lanes_row_kernel<float>(int T, int E);
template <typename real>
hipError_t launch_lanes_row(int T, int E, dim3 grid, hipStream_t s, const RowArgs<real> *args, const BatchItem *items,
                            int tile0, int first0, const void *sched0, PhysArgs ph);
template <>
hipError_t launch_lanes_row<double>(int, int, dim3, hipStream_t, const RowArgs<double> *, const BatchItem *, int, int,
                                    const void *, PhysArgs);
template <>
hipError_t launch_lanes_row<float>(int, int, dim3, hipStream_t, const RowArgs<float> *, const BatchItem *, int, int,
                                   const void *, PhysArgs);
template <typename real>
hipError_t launch_batch_col(int T, int E, bool pad, dim3 grid, hipStream_t s, const ColArgs<real> *args,
                            const BatchItem *items, int tile0, int first0, const void *sched0, PhysArgs ph);
template <>
hipError_t launch_batch_row<double>(int, int, bool, dim3, hipStream_t, const RowArgs<double> *, const BatchItem *, int,
                                   int, const void *, PhysArgs);
template <>
hipError_t launch_batch_row<float>(int, int, bool, dim3, hipStream_t, const RowArgs<float> *, const BatchItem *, int, int,
                                  const void *, PhysArgs);
template <>
hipError_t launch_batch_col<double>(int, int, bool, dim3, hipStream_t, const ColArgs<double> *, const BatchItem *, int,
                                   int, const void *, PhysArgs);
template <>
hipError_t launch_batch_col<float>(int, int, bool, dim3, hipStream_t, const ColArgs<float> *, const BatchItem *, int, int,
                                  const void *, PhysArgs);
// The lift_sym variant of the base-length column kernel (E in {2, 4, 8, 6}).
template <typename real>
hipError_t launch_batch_col_lift(int T, int E, dim3 grid, hipStream_t s, const ColArgs<real> *args,
                                 const BatchItem *items, int tile0, int first0, const void *sched0, PhysArgs ph);
template <>
hipError_t launch_batch_col_lift<double>(int, int, dim3, hipStream_t, const ColArgs<double> *, const BatchItem *, int, int,
                                        const void *, PhysArgs);
template <>
hipError_t launch_batch_col_lift<float>(int, int, dim3, hipStream_t, const ColArgs<float> *, const BatchItem *, int, int,
                                       const void *, PhysArgs);

// Fold-team column kernel (T in {64, 128, 256}, E in {2, 3}); grid.x = one
// block per column.  hipErrorInvalidValue for a shape without an instance.
__host__ __device__ constexpr bool fold_team_shape(int T, int E) {
  return (T == 64 || T == 128 || T == 256) && (E == 2 || E == 3);
}
template <typename real>
hipError_t launch_batch_col_folds(int T, int E, dim3 grid, hipStream_t s, const ColArgs<real> *args,
                                  const BatchItem *items, int tile0, int first0, const void *sched0, PhysArgs ph);
template <>
hipError_t launch_batch_col_folds<double>(int, int, dim3, hipStream_t, const ColArgs<double> *, const BatchItem *, int, int,
                                         const void *, PhysArgs);
template <>
hipError_t launch_batch_col_folds<float>(int, int, dim3, hipStream_t, const ColArgs<float> *, const BatchItem *, int, int,
                                        const void *, PhysArgs);

// Reflecting walls (zk_bc.hip): dst [2ny][2nx] = even extension of src
// [ny][nx]; crop: dst [ny][nx] = the physical quarter of src [2ny][2nx].
hipError_t launch_mirror(const double *src, int nx, int ny, double *dst, hipStream_t s);
hipError_t launch_crop(const double *src, int nx, int ny, double *dst, hipStream_t s);
// Depths of one chunk of layers (zk_bc.hip): dst[i] = y.v[i] for i < kMaxChunkLayers.
struct LayerDepths {
  double v[kMaxChunkLayers];
};
hipError_t launch_set_layer_depths(double *dst, LayerDepths y, hipStream_t s);

// FP64 reductions over base spectra (zk_reduce.hip).  Writes
//   out[0] = sum_k w(kx) Re(conj(a) b),  out[1] = sum_k w(kx) Re(conj(c) d)
// over the stored half spectrum (w = 1 at kx = 0, 2 elsewhere: the full
// spectrum by Hermitian symmetry), in a fixed order.
constexpr int kRedBlocks = 240;
constexpr int kRedThreads = 256;
hipError_t launch_parseval(const cpx<double> *a, const cpx<double> *b, const cpx<double> *c,
                           const cpx<double> *d, int ncols, int ny, double *partial, double *out,
                           hipStream_t s);

}  // namespace zk
