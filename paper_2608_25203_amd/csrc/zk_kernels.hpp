// zk_kernels.hpp -- row-pass and column-pass kernels of the HOS pipeline.
//
// Data layouts (all device memory carved from the caller's workspace):
//   base spectrum   complex<double> [nx/2 / CBB][ny][CBB]: column kx (0 <= kx < nx/2,
//                   the kx = nx/2 Nyquist column is not stored) tiled CBB wide,
//                   index b = ky mode mod ny (b = ny/2 is the Nyquist row, kept 0).
//   mixed field     complex<real> [nx/2 / CBM][rows][CBM]: y physical (rows =
//                   3ny/2 padded, or ny for the base transforms), kx spectral.
//   caller fields   double [ny][nx] row-major.
// A row team is T = nx/8 threads and owns one row; a column team is T = ny/8
// threads and owns one kx column.  Every index below stays inside these
// arrays when the host launches exactly rows/RPB x nprog row blocks and
// ncols/CPB x ntask column blocks (checked on the host).
#pragma once
#include "zk_fft.hpp"
#include "zk_program.hpp"

namespace zk {

constexpr int CBB = 4;  // tile width of base spectra (4 x 16 B = 64 B segments)

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
  const double *pin0, *pin1;
  double *pout0, *pout1;
  const cpx<real> *tw;  // exp(-2 pi i j / N), N = row FFT length
  double kx_scale;      // 2 pi / Lx
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
  const cpx<real> *tw;
  double kx_scale, ky_scale;
  double depth;   // <= 0: deep water
  double inv_kc;  // 1 / kc of the taper
  int taper_on;
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

template <typename real>
__device__ __forceinline__ long long mix_index(int kx, int y, int rows) {
  constexpr int CB = MixTile<real>::CB;
  return ((long long)(kx / CB) * rows + y) * CB + (kx % CB);
}
__device__ __forceinline__ long long base_index(int kx, int b, int ny) {
  return ((long long)(kx / CBB) * ny + b) * CBB + (kx % CBB);
}

// Max over one team of T threads.  Teams of up to 64 threads sit inside one
// wavefront and reduce with lane shuffles; larger teams (one per block) add
// an LDS step across their wavefronts.  red: >= 4 floats of LDS.  Every
// thread of the block must call it.
template <int T>
__device__ __forceinline__ float team_max(float v, float *red) {
  constexpr int W = T < 64 ? T : 64;
#pragma unroll
  for (int o = W / 2; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
  if constexpr (T > 64) {
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    v = red[0];
#pragma unroll
    for (int k = 1; k < T / 64; ++k) v = fmaxf(v, red[k]);
  }
  return v;
}

// Power-of-two scale bringing a magnitude m to [1, 2) (exact; 1 for m == 0).
__device__ __forceinline__ float pow2_scale(float m) {
  return (m > 0.f && m < 3.0e38f) ? ldexpf(1.0f, -ilogbf(m)) : 1.0f;
}

// ---------------------------------------------------------------------------
// Row pass: RPB teams per block, one row each, all running program
// progs[prog0 + blockIdx.y].  Padded rows use E = 12 (N = 3nx/2), base rows
// E = 8 (N = nx).  Row K = nx/2 = 4T spectral columns are stored.
template <typename real, int T, int E>
__global__ __launch_bounds__(256) void row_kernel(RowArgs<real> a) {
  constexpr int N = T * E;
  constexpr int RPB = 256 / T;
  constexpr int L = lds_len(N);
  __shared__ cpx<real> smem[RPB * L];
  __shared__ float red[8];
  const int team = threadIdx.x / T;
  const int t = threadIdx.x % T;
  const int row = blockIdx.x * RPB + team;
  cpx<real> *lds = smem + team * L;
  const RowProg pg = a.progs[a.prog0 + blockIdx.y];

  // Register sets: u = z[].x, v = z[].y (the FFT buffer), then A, o0, o1, o2.
  cpx<real> z[E];
  real R[kRowRegs - 2][E];
#pragma unroll
  for (int e = 0; e < E; ++e) z[e] = {(real)0, (real)0};
#pragma unroll
  for (int s = 0; s < kRowRegs - 2; ++s)
#pragma unroll
    for (int e = 0; e < E; ++e) R[s][e] = (real)0;
  auto reg = [&](auto S, int e) -> real & {
    constexpr int s = decltype(S)::value;
    if constexpr (s == RS_U) return z[e].x;
    else if constexpr (s == RS_V) return z[e].y;
    else return R[s - 2][e];
  };

  for (int i = 0; i < pg.nop; ++i) {
    const RowOp op = a.ops[pg.op0 + i];
    switch (op.code) {
      case OP_LD2: {
        const cpx<real> *Fa = a.mix + (long long)op.fa * a.mix_stride;
        const cpx<real> *Fb = a.mix + (long long)(op.fb >= 0 ? op.fb : 0) * a.mix_stride;
        const bool has_b = op.fb >= 0;
        const bool dxa = op.fla & FL_DX, dxb = op.flb & FL_DX;
        cpx<real> zt[E];
#pragma unroll
        for (int r = 0; r < E; ++r) {
          cpx<real> za = {0, 0}, zb = {0, 0};
          const bool pos = r < 4;
          const bool neg = (r > E - 4) || (r == E - 4 && t > 0);
          if (pos || neg) {
            const int kk = pos ? (t + T * r) : ((E - r) * T - t);
            const long long idx = mix_index<real>(kk, row, a.rows);
            za = Fa[idx];
            if (has_b) zb = Fb[idx];
            const real kxv = (real)(a.kx_scale * kk);
            if (dxa) za = {-kxv * za.y, kxv * za.x};
            if (dxb) zb = {-kxv * zb.y, kxv * zb.x};
            if (neg) {
              za.y = -za.y;
              zb.y = -zb.y;
            }
          }
          z[r] = {za.x, za.y};
          zt[r] = zb;
        }
        // The two real fields share one complex transform; each is scaled by
        // a power of two from its row maximum so that neither drowns in the
        // rounding of the other, and unscaled exactly afterwards.
        float ma = 0.f, mb = 0.f;
#pragma unroll
        for (int r = 0; r < E; ++r) {
          ma = fmaxf(ma, fmaxf(fabsf((float)z[r].x), fabsf((float)z[r].y)));
          mb = fmaxf(mb, fmaxf(fabsf((float)zt[r].x), fabsf((float)zt[r].y)));
        }
        const real sa = (real)pow2_scale(team_max<T>(ma, red));
        const real sb = (real)pow2_scale(team_max<T>(mb, red));
#pragma unroll
        for (int r = 0; r < E; ++r) z[r] = {z[r].x * sa - zt[r].y * sb, z[r].y * sa + zt[r].x * sb};
        team_fft<real, N, E, +1>(z, lds, a.tw, t);
        const real ia = (real)1 / sa, ib = (real)1 / sb;
#pragma unroll
        for (int e = 0; e < E; ++e) z[e] = {z[e].x * ia, z[e].y * ib};
        break;
      }
      case OP_LDP: {
        if constexpr (E != 8) break;  // caller fields have base-length rows only
        const double *pa = op.fa == 0 ? a.pin0 : a.pin1;
        const double *pb = op.fb == 0 ? a.pin0 : a.pin1;
        const long long off = (long long)row * a.nx;
#pragma unroll
        for (int e = 0; e < E; ++e) {
          z[e].x = (real)pa[off + t + T * e];
          z[e].y = op.fb >= 0 ? (real)pb[off + t + T * e] : (real)0;
        }
        break;
      }
      case OP_MOV: {
        with_any(op.a, [&](auto D) {
          with_any(op.b, [&](auto S) {
#pragma unroll
            for (int e = 0; e < E; ++e) reg(D, e) = reg(S, e);
          });
        });
        break;
      }
      case OP_MAC: {
        const real c = (real)op.coef;
        with_out(op.a, [&](auto D) {
          with_in(op.b, [&](auto X) {
            with_in(op.c, [&](auto Y) {
#pragma unroll
              for (int e = 0; e < E; ++e) reg(D, e) += c * reg(X, e) * reg(Y, e);
            });
          });
        });
        break;
      }
      case OP_ZERO: {
        with_any(op.a, [&](auto D) {
#pragma unroll
          for (int e = 0; e < E; ++e) reg(D, e) = (real)0;
        });
        break;
      }
      case OP_BERN: {
        const real eps = (real)op.coef;
#pragma unroll
        for (int e = 0; e < E; ++e) {
          const real S = (real)1 + eps * eps * R[RS_O0 - 2][e];
          const real W = (z[e].x + eps * R[RS_O1 - 2][e]) / S;
          R[RS_O0 - 2][e] = eps * ((real)-0.5 * R[RS_O2 - 2][e] + (real)0.5 * S * W * W);
        }
        break;
      }
      case OP_ST2: {
        real tx[E], ty[E];
        with_any(op.a, [&](auto X) {
#pragma unroll
          for (int e = 0; e < E; ++e) tx[e] = reg(X, e);
        });
        if (op.b != RS_NONE) {
          with_any(op.b, [&](auto Y) {
#pragma unroll
            for (int e = 0; e < E; ++e) ty[e] = reg(Y, e);
          });
        } else {
#pragma unroll
          for (int e = 0; e < E; ++e) ty[e] = (real)0;
        }
        float mx = 0.f, my = 0.f;
#pragma unroll
        for (int e = 0; e < E; ++e) {
          mx = fmaxf(mx, fabsf((float)tx[e]));
          my = fmaxf(my, fabsf((float)ty[e]));
        }
        const real sx = (real)pow2_scale(team_max<T>(mx, red));
        const real sy = (real)pow2_scale(team_max<T>(my, red));
#pragma unroll
        for (int e = 0; e < E; ++e) z[e] = {tx[e] * sx, ty[e] * sy};
        team_fft<real, N, E, -1>(z, lds, a.tw, t);
        __syncthreads();
#pragma unroll
        for (int e = 0; e < E; ++e) lds[lpad(t + T * e)] = z[e];
        __syncthreads();
        cpx<real> *Fa = a.mix + (long long)op.fa * a.mix_stride;
        cpx<real> *Fb = a.mix + (long long)(op.fb >= 0 ? op.fb : 0) * a.mix_stride;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int k = t + T * q;
          const cpx<real> zk = lds[lpad(k)];
          const cpx<real> zm = lds[lpad(k == 0 ? 0 : N - k)];
          const long long idx = mix_index<real>(k, row, a.rows);
          const real hx = (real)0.5 / sx, hy = (real)0.5 / sy;
          Fa[idx] = {hx * (zk.x + zm.x), hx * (zk.y - zm.y)};
          if (op.fb >= 0) Fb[idx] = {hy * (zk.y + zm.y), -hy * (zk.x - zm.x)};
        }
        break;
      }
      case OP_STP: {
        if constexpr (E != 8) break;
        double *po = op.fa == 0 ? a.pout0 : a.pout1;
        const long long off = (long long)row * a.nx;
        with_any(op.a, [&](auto X) {
#pragma unroll
          for (int e = 0; e < E; ++e) po[off + t + T * e] = (double)reg(X, e);
        });
        break;
      }
      default:
        break;
    }
  }
}

// ---------------------------------------------------------------------------
// Fourier symbols at (kx, b) of the base band.
__device__ __forceinline__ double filt1(int m, int n) {
  const double th = 2.0 * M_PI * (double)m / (double)n;
  return (5.0 + 4.0 * cos(th) - cos(2.0 * th)) * 0.125;
}

// symbol s at kx = col, ky mode my, |k| = kk, tanh(|k| d) = th
template <typename real>
__device__ __forceinline__ cpx<double> symval(uint32_t s, int col, int my, double kk, double th,
                                              const ColArgs<real> &a) {
  double f = 1.0;
  const int l = s & SYM_LMASK;
  if (l) {
    double p = kk;
    for (int i = 1; i < l; ++i) p *= kk;
    f = (l & 1) ? p * th : p;
  }
  if (s & SYM_FILT) f *= filt1(col, a.nx) * filt1(my, a.ny);
  if ((s & SYM_TAPER) && a.taper_on) {
    const double r2 = kk * kk * a.inv_kc * a.inv_kc;
    const double r4 = r2 * r2;
    f *= exp(-(r4 * r4));
  }
  if (s & SYM_IKY) return {0.0, f * (a.ky_scale * my)};
  return {f, 0.0};
}

// Column pass: CPB teams per block, one kx column each, all running task
// tasks[task0 + blockIdx.y].  Padded columns use E = 12 (N = 3ny/2), base
// columns E = 8 (N = ny).  Thread t owns base-band rows b = t + T q, q < 8.
template <typename real, int T, int E>
__global__ __launch_bounds__(256) void col_kernel(ColArgs<real> a) {
  constexpr int N = T * E;
  constexpr int CPB = (256 / T < 4) ? 256 / T : 4;
  constexpr int L = lds_len(N);
  constexpr int CB = MixTile<real>::CB;
  __shared__ cpx<real> smem[CPB * L];
  const int team = threadIdx.x / T;
  const int t = threadIdx.x % T;
  const int col = blockIdx.x * CPB + team;
  cpx<real> *lds = smem + team * L;
  const ColTask task = a.tasks[a.task0 + blockIdx.y];
  const int ny = a.ny;

  double kk[8], th[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int b = t + T * q;
    const int my = (b < ny / 2) ? b : b - ny;
    const double kx = a.kx_scale * col, ky = a.ky_scale * my;
    kk[q] = sqrt(kx * kx + ky * ky);
    th[q] = a.depth > 0.0 ? tanh(kk[q] * a.depth) : 1.0;
  }
  auto my_of = [&](int q) {
    const int b = t + T * q;
    return (b < ny / 2) ? b : b - ny;
  };

  cpx<double> X[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) X[q] = {0.0, 0.0};
  if (task.fwd >= 0) {
    const cpx<real> *F = a.mix + (long long)task.fwd * a.mix_stride;
    cpx<real> v[E];
#pragma unroll
    for (int r = 0; r < E; ++r) v[r] = F[mix_index<real>(col, t + T * r, a.rows)];
    team_fft<real, N, E, -1>(v, lds, a.tw, t);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int src = (E == 12 && q >= 4) ? q + 4 : q;
      const cpx<double> s = symval(task.fwd_sym, col, my_of(q), kk[q], th[q], a);
      const cpx<double> x = {(double)v[src].x * task.fwd_coef, (double)v[src].y * task.fwd_coef};
      X[q] = {x.x * s.x - x.y * s.y, x.x * s.y + x.y * s.x};
    }
    if (t == 0) X[4] = {0.0, 0.0};  // ky Nyquist row
  }

  for (int o = 0; o < task.no; ++o) {
    const ColOut out = a.outs[task.o0 + o];
    cpx<double> acc[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) acc[q] = {0.0, 0.0};
    for (int i = 0; i < out.nt; ++i) {
      const ColTerm tm = a.terms[out.t0 + i];
      cpx<double> s0[8];
      if (tm.src >= 0) {
        const cpx<double> *B = a.base + (long long)tm.src * a.base_stride;
#pragma unroll
        for (int q = 0; q < 8; ++q) s0[q] = B[base_index(col, t + T * q, ny)];
      } else {
#pragma unroll
        for (int q = 0; q < 8; ++q) s0[q] = X[q];
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        cpx<double> s = symval(tm.sym, col, my_of(q), kk[q], th[q], a);
        s = {s.x * tm.coef, s.y * tm.coef};
        acc[q].x += s0[q].x * s.x - s0[q].y * s.y;
        acc[q].y += s0[q].x * s.y + s0[q].y * s.x;
      }
    }
    if (t == 0) acc[4] = {0.0, 0.0};
    if (out.dst_base >= 0) {
      cpx<double> *B = a.base + (long long)out.dst_base * a.base_stride;
#pragma unroll
      for (int q = 0; q < 8; ++q) B[base_index(col, t + T * q, ny)] = acc[q];
    }
    if (out.dst_mixed >= 0) {
      const double lc = out.lift_coef;
      cpx<real> z[E];
#pragma unroll
      for (int r = 0; r < E; ++r) {
        int q = -1;
        if (E == 8) q = r;
        else if (r < 4) q = r;
        else if (r >= 8) q = r - 4;
        z[r] = q >= 0 ? cpx<real>{(real)(acc[q].x * lc), (real)(acc[q].y * lc)} : cpx<real>{0, 0};
      }
      team_fft<real, N, E, +1>(z, lds, a.tw, t);
      cpx<real> *F = a.mix + (long long)out.dst_mixed * a.mix_stride;
#pragma unroll
      for (int r = 0; r < E; ++r) F[mix_index<real>(col, t + T * r, a.rows)] = z[r];
    }
  }
}

// launch wrappers (defined in the per-precision instantiation units)
template <typename real>
hipError_t launch_row(const RowArgs<real> &a, int T, int E, int nblocks, int nprog, hipStream_t s);
template <typename real>
hipError_t launch_col(const ColArgs<real> &a, int T, int E, int nblocks, int ntask, hipStream_t s);
template <>
hipError_t launch_row<double>(const RowArgs<double> &a, int T, int E, int nblocks, int nprog, hipStream_t s);
template <>
hipError_t launch_row<float>(const RowArgs<float> &a, int T, int E, int nblocks, int nprog, hipStream_t s);
template <>
hipError_t launch_col<double>(const ColArgs<double> &a, int T, int E, int nblocks, int ntask, hipStream_t s);
template <>
hipError_t launch_col<float>(const ColArgs<float> &a, int T, int E, int nblocks, int ntask, hipStream_t s);

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
