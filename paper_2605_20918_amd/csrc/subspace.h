// Internal: Fermi operator inside the Krylov subspace by a pole expansion.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

#include "css_common.h"

namespace css {

// F (nT x b, row-major, nT = v*b) = g f(T) E_1 B_0 for the block tridiagonal T
// given by A_j, B_j (ld x ld padded); sums[0] = trace_K, sums[1] = E_K (device).
// Synchronises the stream once (spectral bound -> number of poles).
css_status subspace_fermi_poles(const double* A, const double* B, int v, int b, int ld, const int* counts,
                                double mu, double kT, double g, double* F, double* sums, void* ws, size_t ws_bytes,
                                int* npoles_out, hipStream_t s);
// Workspace of subspace_fermi_poles for at most max_poles poles (0: the most the
// expansion ever uses, 257).
size_t pole_workspace_bytes(int v, int b, int max_poles = 0);
// Gershgorin bounds of T (every Ritz value lies in [lo, hi]); host outputs,
// synchronises the stream. ws: at least 2 v b + 16 doubles (the pole workspace is).
css_status subspace_spectral_bounds(const double* A, const double* B, int v, int b, int ld, void* ws, size_t ws_bytes,
                                    double* lo, double* hi, hipStream_t s);

}  // namespace css
