// Adaptive face coarse DOFs (Section 3.3), host side (adaptive.cpp).
#pragma once

#include "internal.h"

namespace bddc {

// One face problem in the jump space of its m shared nodes G (row-major
// m x m matrices in the order of G).
struct FaceInput {
    int m;
    const double *Hs, *Ht;       // Schur complements of S_s, S_t onto G
    const double *Ks, *Kt;       // S_s(G, G), S_t(G, G)
    const double *Ds, *Dt;       // interface weights of s and t on G
    bool float_s, float_t;       // subdomain without Dirichlet nodes
    int nb;                      // shared coarse DOFs
    const double *B;             // their rows over G (nb x m)
    int nf;                      // the face's own nodes
    const int32_t *fpos;         // their positions in G
};

struct FaceOutput {
    std::vector<double> lam;                 // eigenvalues of the pencil, descending
    std::vector<std::vector<double>> rows;   // new rows over the face nodes (orthonormal)
};

struct AdaptStats {
    int faces = 0, added = 0;
    double lam_max = 0.0, seconds = 0.0;
};

// lobpcg_it > 0: the max_rows largest pairs by LOBPCG with at most that many
// iterations (out.lam then holds only those Ritz values), else the whole
// pencil by a dense symmetric eigensolver.
int face_rows(const FaceInput &in, double tau, int max_rows, FaceOutput &out, int lobpcg_it = 0,
              int *lobpcg_iters = nullptr);

// Every level-1 face of `st`: Schur complements on the device (S_i in the
// swept local matrices d_K at k_off), the pencils on the host; the new rows
// are returned as coarse DOFs of kind 3.
int adaptive_faces(const Structure &st, const double *d_K, const std::vector<int64_t> &k_off, double tau,
                   int max_per_face, int lobpcg_it, int32_t *d_status, hipStream_t s, std::vector<CoarseDof> &extra,
                   AdaptStats &stats, std::string &err);

// Every level-2 face (three levels): S2 holds each subregion's Schur
// complement on its level-2 interface (row-major nB x nB, the order of
// SubregionHost::L after the interior ids); floating marks subregions whose
// subdomains all lack Dirichlet nodes.  New rows are returned as level-3 DOFs.
int adaptive_level2(const Structure &st, const std::vector<std::vector<double>> &S2,
                    const std::vector<char> &floating, double tau, int max_per_face, int lobpcg_it,
                    std::vector<Level3Dof> &extra, AdaptStats &stats, std::string &err);

}  // namespace bddc
