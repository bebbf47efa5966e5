// Reads one face problem of the adaptive coarse-space selection from stdin,
// runs the library's host routine on it and prints the eigenvalues and the
// new rows (built with sanitizers by tests/test_host_linalg.py).
#include <cstdio>
#include <vector>

#include "adaptive.h"

int main() {
    int m, max_rows, fs, ft, nb, nf;
    double tau;
    if (std::scanf("%d %lf %d %d %d %d %d", &m, &tau, &max_rows, &fs, &ft, &nb, &nf) != 7) return 2;
    auto read = [](std::vector<double> &v, size_t n) {
        v.resize(n);
        for (size_t i = 0; i < n; ++i)
            if (std::scanf("%lf", &v[i]) != 1) return false;
        return true;
    };
    std::vector<double> Hs, Ht, Ks, Kt, Ds, Dt, B;
    const size_t mm = (size_t)m * m;
    if (!read(Hs, mm) || !read(Ht, mm) || !read(Ks, mm) || !read(Kt, mm) || !read(Ds, m) || !read(Dt, m) ||
        !read(B, (size_t)nb * m))
        return 2;
    std::vector<int32_t> fpos(nf);
    for (int q = 0; q < nf; ++q)
        if (std::scanf("%d", &fpos[q]) != 1) return 2;
    bddc::FaceInput in{m, Hs.data(), Ht.data(), Ks.data(), Kt.data(), Ds.data(), Dt.data(), fs != 0, ft != 0, nb,
                       B.data(), nf, fpos.data()};
    bddc::FaceOutput out;
    const int rc = bddc::face_rows(in, tau, max_rows, out);
    if (rc) return 3;
    std::printf("%d\n", (int)out.lam.size());
    for (double v : out.lam) std::printf("%.17g\n", v);
    std::printf("%d\n", (int)out.rows.size());
    for (const auto &r : out.rows)
        for (double v : r) std::printf("%.17g\n", v);
    return 0;
}
