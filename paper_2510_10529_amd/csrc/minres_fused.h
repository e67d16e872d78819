// Fused MINRES passes (minres_fused.hip).
#pragma once

#include "internal.h"

namespace invdft {

struct FusedWork {
  double *partG, *partD, *G, *d1, *d2;
};

size_t fused_work_bytes(int64_t N);
FusedWork fused_layout(void* base, int64_t N);

// G = Psi^T Y (k0 x k), d1 = col-dot(Z, Y), d2 = col-dot(Z, R1)
template <typename T>
fe_status minres_pass_a(const T* Psi, int k0, const T* Y, const T* Z, const T* R1, int k, int64_t N, FusedWork& fw,
                        hipStream_t s);
}  // namespace invdft
