// Small dense symmetric eigensolver (host): cyclic Jacobi rotations.
// Used for the Lanczos tridiagonal T_m (m <= 64) to get the extreme Ritz
// values and the last component of the top Ritz vector.
#pragma once
#include <cmath>
#include <vector>

namespace ppeig {

// a: m x m symmetric, row-major (destroyed).  On return w holds the
// eigenvalues (unsorted) and column c of v (v[r*m + c]) the eigenvector of w[c].
inline void jacobi_eig(int m, std::vector<double> &a, std::vector<double> &w, std::vector<double> &v)
{
    v.assign((size_t)m * m, 0.0);
    for (int i = 0; i < m; ++i) v[(size_t)i * m + i] = 1.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < m; ++j) {
                const double x = a[(size_t)i * m + j] * a[(size_t)i * m + j];
                tot += x;
                if (i != j) off += x;
            }
        if (off <= 1e-32 * tot || off == 0.0) break;
        for (int p = 0; p < m - 1; ++p) {
            for (int q = p + 1; q < m; ++q) {
                const double apq = a[(size_t)p * m + q];
                if (apq == 0.0) continue;
                const double app = a[(size_t)p * m + p], aqq = a[(size_t)q * m + q];
                // rotation angle: tan(2 phi) = 2 apq / (aqq - app), smaller root for t
                const double th = (aqq - app) / (2.0 * apq);
                const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
                const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < m; ++k) {  // columns p, q
                    const double akp = a[(size_t)k * m + p], akq = a[(size_t)k * m + q];
                    a[(size_t)k * m + p] = c * akp - s * akq;
                    a[(size_t)k * m + q] = s * akp + c * akq;
                }
                for (int k = 0; k < m; ++k) {  // rows p, q
                    const double apk = a[(size_t)p * m + k], aqk = a[(size_t)q * m + k];
                    a[(size_t)p * m + k] = c * apk - s * aqk;
                    a[(size_t)q * m + k] = s * apk + c * aqk;
                }
                for (int k = 0; k < m; ++k) {
                    const double vkp = v[(size_t)k * m + p], vkq = v[(size_t)k * m + q];
                    v[(size_t)k * m + p] = c * vkp - s * vkq;
                    v[(size_t)k * m + q] = s * vkp + c * vkq;
                }
            }
        }
    }
    w.resize(m);
    for (int i = 0; i < m; ++i) w[i] = a[(size_t)i * m + i];
}

}  // namespace ppeig
