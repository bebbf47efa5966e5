// Host check of the library's symmetric eigensolver (hostla.cpp): reads n and
// a row-major n x n matrix from stdin, prints the eigenvalues and then the
// row-major eigenvector matrix, one number per line.
#include <cstdio>
#include <vector>

#include "internal.h"

int main() {
    int n;
    if (std::scanf("%d", &n) != 1 || n < 0) return 1;
    std::vector<double> a((size_t)n * n);
    for (auto &x : a)
        if (std::scanf("%lf", &x) != 1) return 1;
    std::vector<double> w, v;
    bddc::sym_eig(a, n, w, v);
    for (double x : w) std::printf("%.17g\n", x);
    for (double x : v) std::printf("%.17g\n", x);
    return 0;
}
