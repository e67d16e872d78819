// Fused MINRES passes (minres_fused.hip).
#pragma once

#include "internal.h"

namespace invdft {

struct FusedWork {
  double *partG, *partD;  // per-workgroup partial sums (shared by passes A and B)
  double *G, *d1, *d2;    // pass A: G1 = Psi^T y, z.y, z.r1
  double *G2, *d;         // pass B: G2 = Psi^T u, r.u
};

size_t fused_work_bytes(int64_t N);
FusedWork fused_layout(void* base, int64_t N);

// G = Psi^T Y (k0 x k), d1 = col-dot(Z, Y), d2 = col-dot(Z, R1)
template <typename T>
fe_status minres_pass_a(const T* Psi, int k0, const T* Y, const T* Z, const T* R1, int k, int64_t N, FusedWork& fw,
                        hipStream_t s);
// r = Y - Psi G1 - c1 R1 - c2 R2 (over R1), u = D^{-1} r (over Y), G2 = Psi^T u, d = r.u;
// G1 is fw.G from pass A, c1 and c2 the per-column MINRES coefficients in st
template <typename T>
fe_status minres_pass_b(const T* Psi, int k0, T* Y, T* R1, const T* R2, const double* st, const double* dinv, int k,
                        int64_t N, FusedWork& fw, hipStream_t s);

// z = U - Psi G2 (over U; zero for converged columns), then the MINRES direction and
// solution update w_new = (Zold / beta_old - oldeps W1 - delta W2) / gamma (over W1),
// X += phi w_new, with the scalars of st (columns with 1/gamma = 0 are left unchanged)
template <typename T>
fe_status minres_pass_c(const T* Psi, int k0, T* U, const T* Zold, T* W1, const T* W2, T* X, const double* st, int k,
                        int64_t N, FusedWork& fw, hipStream_t s);
}  // namespace invdft
