// Host FP64 minimax Laplace quadrature (see quadrature.cpp).
#pragma once

namespace ltmp2 {

// R_floor(n): smallest R at which an n-point fit is computed.
double quad_r_floor(int n);

// tau, w [n] for 1/x on [x_min, x_max]; 0 on success, 1 bad input, 2 no convergence.
int minimax_quadrature(double x_min, double x_max, int n, double* tau, double* w, double* delta);

// `steps` Remez passes from the proposal in (tau, w); certified = 1 if the
// 2n + 1 alternation levels agree to cert_tol relative.
int remez_polish(double x_min, double x_max, int n, int steps, double cert_tol, double* tau,
                 double* w, double* delta, int* certified);

// Minimax fits on [1, max(R[k], R_floor)] for ascending R[0..count) by one
// continuation sweep: alpha, beta [count][n] (unit interval), delta [count].
int quadrature_table(int n, int count, const double* R, double* alpha, double* beta,
                     double* delta);

}  // namespace ltmp2
