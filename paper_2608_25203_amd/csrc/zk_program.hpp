// zk_program.hpp -- schedule records shared by the host planner and the kernels.
//
// One right-hand-side evaluation is a chain of two kinds of launches:
//
//  * row passes: one team of T = n/8 threads per padded (or base) grid row.
//    A row program is a short list of RowOps: inverse x-FFT of pairs of
//    "mixed" fields (y physical, kx spectral) into physical row values held in
//    registers, pointwise sums of products, forward x-FFT of pairs of results
//    back to mixed fields.  Pointwise work never leaves registers.
//  * column passes: one team per kx column.  A ColTask optionally runs the
//    forward y-FFT of one mixed field, truncates it to the base band and
//    tapers it (the fold of the dealiased product), then produces ColOuts:
//    linear combinations of that result and stored base-band spectra, each
//    multiplied by a Fourier symbol, stored as a base spectrum and/or
//    zero-padded and inverse y-FFT'd into a mixed field (the lift).
#pragma once
#include <stdint.h>

namespace zk {

// ---- row programs -------------------------------------------------------
enum RowCode : uint8_t {
  OP_LD2 = 1,  // u + i v <- inverse x-FFT of (F_a, F_b) mixed rows (Hermitian ext.)
  OP_LDP = 2,  // u, v <- physical rows of caller fields (base grid)
  OP_MOV = 3,  // A <- R[b] (a = A)
  OP_MAC = 4,  // R[a] += coef * R[b] * R[c], a in o0..o2, b, c in u, v, A
  OP_ZERO = 5, // o0, o1, o2 <- 0
  OP_BERN = 6, // o0 <- Bernoulli term from o0 = |grad eta|^2, o1 = grad eta.grad psi,
               //       o2 = |grad psi|^2, u = G psi; coef = eps
  OP_ST2 = 7,  // forward x-FFT of R[a] + i R[b]; split; store kx < nx/2 to mixed fa, fb
  OP_STP = 8   // physical row of R[a] -> caller field slot fa, plane fb >= 0 of it (base grid)
};

// register sets of a row team (each E values per thread)
enum RowReg : uint8_t { RS_U = 0, RS_V = 1, RS_A = 2, RS_O0 = 3, RS_O1 = 4, RS_O2 = 5, RS_NONE = 255 };
constexpr int kRowRegs = 6;

enum RowFlag : uint8_t { FL_DX = 1 };  // multiply the spectrum by i*kx before the inverse FFT

struct RowOp {
  uint8_t code, a, b, c;
  uint8_t fla, flb, pad0, pad1;
  int32_t fa, fb;  // mixed-field ids, or caller-field slots for LDP/STP; -1 = none
  double coef;
};

struct RowProg {
  int32_t op0, nop;
  int32_t shape1;  // 1 + the program's compiled shape (zk_row_shapes.hpp), or 0: interpreted
  int32_t pad_;
};

// ---- column tasks -------------------------------------------------------
// Fourier symbol bits; the symbol is the product of the selected factors.
enum SymBits : uint32_t {
  SYM_LMASK = 0xF,   // L_l(k) = |k|^l (tanh(|k| d) if l odd), l = bits & 0xF
  SYM_IKY = 0x10,    // i * ky
  SYM_FILT = 0x20,   // state filter A(k)
  SYM_TAPER = 0x40,  // taper exp(-(|k|/kc)^8) (only if the taper option is on)
  SYM_IF = 0x80      // coefficient (bits >> SYM_IF_SHIFT) & 7 of the exact linear flow
                     // and its constant-forcing response (Sec. 3.4, eq:lin_prop,
                     // eq:if_ab2_eta, eq:if_ab2_psi): 0 cos(w dt), 1 G0 sin(w dt)/w,
                     // 2 g sin(w dt)/w, 3 sin(w dt)/w, 4 (1-cos(w dt))/g, 5 (1-cos(w dt))/G0
};
constexpr int SYM_IF_SHIFT = 8;
constexpr uint32_t SYM_INVG0 = 0x800;  // 1 / G0 off k = 0, 0 at k = 0 (inverse DNO seed and update)
// Bulk velocity at a depth layer (Sec. on finite-depth kernels and coupling
// taper); these act only through ColOut.lift_sym:
constexpr uint32_t SYM_COUPLE = 0x1000;   // prod_a exp(-(|k_a| / (kNyq_a / 2))^8)
constexpr uint32_t SYM_LAYER_C = 0x2000;  // C_i of layer i of the chunk (eq:Ci, eq:CiSi_stable)
constexpr uint32_t SYM_LAYER_S = 0x4000;  // S_i of layer i of the chunk (eq:Si, eq:CiSi_stable)
constexpr int SYM_LAYER_SHIFT = 16;       // bits 16..19: i, the layer's index in its chunk
constexpr int kMaxChunkLayers = 16;       // depth layers lifted per column/row launch pair
constexpr int kIfCoefs = 6;

struct ColTerm {
  int32_t src;   // base-spectrum id, or -1 = the task's folded sum X
  uint32_t sym;
  double coef;
};

struct ColOut {
  int32_t dst_base;   // base-spectrum id to store the combination, or -1
  int32_t dst_mixed;  // mixed-field id to lift the combination into, or -1
  int32_t t0, nt;     // terms [t0, t0 + nt)
  double lift_coef;   // extra factor applied before the lift (1/N)
  uint32_t lift_sym;  // depth-lift factors (SYM_COUPLE, SYM_LAYER_*) applied to the lifted copy only, or 0
  uint32_t pad_;
};

// A column task folds up to kMaxFolds mixed fields (forward y-FFT, band
// truncation), each times its symbol and scale, into one sum X that its
// outputs' terms may use (src = -1).
constexpr int kMaxFolds = 3;
struct ColTask {
  int32_t fwd[kMaxFolds];       // mixed-field ids to fold, or -1
  uint32_t fwd_sym[kMaxFolds];  // symbol applied to each folded field
  double fwd_coef[kMaxFolds];   // scale applied to each folded field
  int32_t o0, no;               // outputs [o0, o0 + no)
};

}  // namespace zk
