// Scalar part of the three retractions of Sec. 6 (host, FP64).  Each
// retraction scales component l of w = u + t xi by a factor sigma_l fixed by
// the component norms a_l = ||w_l||^2 alone; these functions compute the
// factors.  Storage index i holds l = F - i (i = 0 .. 2F).
//
// Plain C++ with no HIP dependency: the library calls them between its norm
// and scaling kernels, and they also build on their own (with sanitizers) for
// host-only checks.
#pragma once

namespace gpe {

enum SigmaStatus { SIGMA_OK = 0, SIGMA_DOMAIN = 2 };

// Projective retraction (Sec. 6.1): with f1 < M < f2 the lowest and highest l
// carrying mass, r is the zero of the increasing h1 on (1/(f1-M), 1/(f2-M))
// and sigma_l = 1 / (sqrt(s) (1 - (l-M) r)) on [f1, f2], 0 outside.
// SIGMA_DOMAIN if w is outside Omega (no mass on one side of M).
int sigma_projective(int F, double M, const double* a, double* sig);

// Orthogonal retraction (Sec. 6.2): sigma_l = sqrt(r^l / sum_k a_k r^k), r the
// positive zero of h2.  SIGMA_DOMAIN outside Omega.
int sigma_orthogonal(int F, double M, const double* a, double* sig);

// Closed-form retraction (Sec. 6.3, eq. retract3).  SIGMA_DOMAIN outside S.
int sigma_closed(int F, double M, const double* a, double* sig);

}  // namespace gpe
