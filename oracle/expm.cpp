/*
 * Matrix exponential by scaling and squaring with diagonal Pade
 * approximants (Higham 2005, SIAM J. Matrix Anal. Appl. 26, 1179): pick the
 * lowest degree m in {3, 5, 7, 9} whose threshold theta_m bounds the 1-norm,
 * otherwise scale by 2^-s to bring the norm under theta_13, apply the
 * degree-13 approximant and square s times.  The approximant is
 * r_m(A) = q_m(A)^-1 p_m(A), p_m(x) = sum_j b_j x^j, q_m(x) = p_m(-x),
 * b_j = (2m - j)! m! / ((2m)! j! (m - j)!), evaluated by plain powers and a
 * Gaussian-elimination solve.  Test infrastructure only (CPU oracle).
 */
#include <cmath>
#include <cstring>
#include "oracle_internal.h"

namespace orc {

static const int NMAX = 8;

static void matmul(int n, const double* A, const double* B, double* C) {
    double T[NMAX * NMAX];
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            double s = 0.0;
            for (int k = 0; k < n; ++k) s += A[i * n + k] * B[k * n + j];
            T[i * n + j] = s;
        }
    std::memcpy(C, T, sizeof(double) * n * n);
}

static double factorial(int k) {
    double f = 1.0;
    for (int i = 2; i <= k; ++i) f *= i;
    return f;
}

static double pade_coef(int m, int j) {
    return factorial(2 * m - j) * factorial(m) / (factorial(2 * m) * factorial(j) * factorial(m - j));
}

/* Solve Q X = P for X (n x n), Gaussian elimination with partial pivoting. */
static int solve(int n, const double* Q, const double* P, double* X) {
    double A[NMAX][2 * NMAX];
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            A[i][j] = Q[i * n + j];
            A[i][n + j] = P[i * n + j];
        }
    for (int col = 0; col < n; ++col) {
        int piv = col;
        for (int i = col + 1; i < n; ++i)
            if (std::fabs(A[i][col]) > std::fabs(A[piv][col])) piv = i;
        if (A[piv][col] == 0.0) return -1;
        if (piv != col)
            for (int j = 0; j < 2 * n; ++j) std::swap(A[piv][j], A[col][j]);
        for (int i = col + 1; i < n; ++i) {
            double f = A[i][col] / A[col][col];
            for (int j = col; j < 2 * n; ++j) A[i][j] -= f * A[col][j];
        }
    }
    for (int j = 0; j < n; ++j)
        for (int i = n - 1; i >= 0; --i) {
            double s = A[i][n + j];
            for (int k = i + 1; k < n; ++k) s -= A[i][k] * X[k * n + j];
            X[i * n + j] = s / A[i][i];
        }
    return 0;
}

static int pade(int n, int m, const double* A, double* R) {
    double P[NMAX * NMAX], Q[NMAX * NMAX], Ak[NMAX * NMAX];
    std::memset(P, 0, sizeof(P));
    std::memset(Q, 0, sizeof(Q));
    for (int i = 0; i < n; ++i) {
        P[i * n + i] = pade_coef(m, 0);
        Q[i * n + i] = pade_coef(m, 0);
    }
    std::memcpy(Ak, A, sizeof(double) * n * n);
    for (int j = 1; j <= m; ++j) {
        double b = pade_coef(m, j);
        double sgn = (j % 2) ? -1.0 : 1.0;
        for (int k = 0; k < n * n; ++k) {
            P[k] += b * Ak[k];
            Q[k] += sgn * b * Ak[k];
        }
        if (j < m) matmul(n, Ak, A, Ak);
    }
    return solve(n, Q, P, R);
}

int expm(int n, const double* A, double* E) {
    if (n < 1 || n > NMAX) return -1;
    double norm = 0.0;
    for (int j = 0; j < n; ++j) {
        double s = 0.0;
        for (int i = 0; i < n; ++i) s += std::fabs(A[i * n + j]);
        if (s > norm) norm = s;
    }
    if (!std::isfinite(norm)) {
        for (int k = 0; k < n * n; ++k) E[k] = NAN;
        return -1;
    }
    const int degs[4] = {3, 5, 7, 9};
    const double theta[4] = {1.495585217958292e-2, 2.539398330063230e-1, 9.504178996162932e-1,
                             2.097847961257068e0};
    for (int k = 0; k < 4; ++k)
        if (norm <= theta[k]) return pade(n, degs[k], A, E);
    const double theta13 = 5.371920351148152e0;
    int s = (int)std::ceil(std::log2(norm / theta13));
    if (s < 0) s = 0;
    double As[NMAX * NMAX];
    double scale = std::ldexp(1.0, -s);
    for (int k = 0; k < n * n; ++k) As[k] = A[k] * scale;
    if (pade(n, 13, As, E) != 0) return -1;
    for (int i = 0; i < s; ++i) matmul(n, E, E, E);
    return 0;
}

}  // namespace orc

extern "C" int or_expm(int n, const double* A, double* E) { return orc::expm(n, A, E); }
