// Optional per-kernel timing with HIP events recorded on the launching
// stream.  Disabled by default (the hooks are then two branches); when
// enabled, every hooked launch is bracketed by a pair of events from a fixed
// pool and rpc_profile_read sums their elapsed times per kernel class.
// Process-global and not thread-safe: for benchmarking only.
#pragma once
#include <hip/hip_runtime.h>

namespace prof {
enum Kind {
  KERNEL_COLS = 0,  // distance product + exp (kernel columns)
  SCHUR = 1,        // W -= F F_S^T
  SOLVE = 2,        // G = W L^{-T}, F write, residual-diagonal downdate
  PIVOT = 3,        // residual quantisation, CDF draw / argmax
  ACCEPT = 4,       // pivot block H and Algorithm 3
  DEGREES = 5,      // c, d~, w, q~
  GRAM = 6,         // the N-long Gram partial products
  SMALL = 7,        // r x r work: Gram reduction and finish, Cholesky, inner product
  FORM_U = 8,       // U = D~^{-1} F R^{-1} V and signs
  NYSTROM = 9,
  EIG = 10,         // top-nev eigenpairs of the r x r inner matrix
  SUR_TRAIN = 11,   // one surrogate training step
  SUR_INFER = 12,   // surrogate forward pass
  NKIND = 13
};
bool enabled();
void begin(int kind, hipStream_t st);
void end(int kind, hipStream_t st);
}  // namespace prof
