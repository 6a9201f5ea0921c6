// Host-only parameter selection of libqsw (params.cpp): theta_m tables and
// the choice of Taylor degree m and scaling s.
#pragma once

#include <stdint.h>

#include "../../include/qsw.h"

namespace qsw {

// theta_m for m = 1..55 of the truncated-Taylor backward-error bound with
// unit roundoff 2^-53 (prec = QSW_PREC_DOUBLE) or 2^-24 (QSW_PREC_SINGLE and
// QSW_PREC_FP32).
double theta_of(int m, int prec);

// Unit roundoff of the precision.
double tol_of(int prec);

// Largest Taylor degree of the precision (55; 20 for QSW_PREC_FP32).
int mmax_of(int prec);

// m and s for exp(t L); d = NULL uses ||L||_1 only, else d[p], p = 2..9.
// switch313: apply Al-Mohy and Higham's switch to the 1-norm rule for small
// ||tL||_1 (false: the alpha_p rule whenever d is given).
qsw_status_t select_params_impl(double norm1, const double *d, double t, int n0, int prec,
                                int *m_out, int *s_out, bool switch313 = true);

}  // namespace qsw
