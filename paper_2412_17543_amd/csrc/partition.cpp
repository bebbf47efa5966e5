// Mesh, partition and coarse-space bookkeeping on the host (Section 3.1 and
// Section 3.2 of Hanek, Papez & Sistek, arXiv 2412.17543).
//
// Reading of the coarse-DOF selection (the paper only says "function values at
// selected interface nodes (corners) and arithmetic averages across faces and
// edges"):
//   S(n)  = sorted set of subdomains owning kept elements around node n, for
//           every node touched by a kept element (Dirichlet nodes included);
//   glob  = 6-connected set of nodes with |S| >= 2 and identical S;
//   face  = glob with |S| = 2, coarse DOF = mean over its free nodes;
//   corner= free node with |S| >= 3 whose glob is a single node or that has at
//           most one axis neighbour in its glob, and none of whose axis
//           neighbours has a strictly larger S;
//   edge  = (optional) glob with |S| >= 3, mean over its free non-corner nodes.
// Three levels: subdomains act as elements of the coarse problem and are
// grouped into subregions; S2(c) = subregions owning coarse DOF c; level-2
// globs are level-2 interface DOFs with equal S2 linked through a shared
// subdomain; level-2 faces (|S2| = 2) get averages, level-2 corners are
// level-1 corners with |S2| >= 3 passing the same endpoint/superset test with
// "shares a subdomain" as neighbour relation; level-2 weights are 1/|S2|.
#include <algorithm>
#include <cmath>
#include <map>
#include <numeric>

#include "internal.h"

namespace bddc {

namespace {

struct SubSet {
    uint8_t n = 0;
    int32_t s[8];
    bool operator==(const SubSet &o) const {
        if (n != o.n) return false;
        for (int i = 0; i < n; ++i)
            if (s[i] != o.s[i]) return false;
        return true;
    }
    void insert(int32_t v) {
        int i = 0;
        while (i < n && s[i] < v) ++i;
        if (i < n && s[i] == v) return;
        for (int j = n; j > i; --j) s[j] = s[j - 1];
        s[i] = v;
        ++n;
    }
    // true when *this is a strict subset of o
    bool strict_subset_of(const SubSet &o) const {
        if (o.n <= n) return false;
        int j = 0;
        for (int i = 0; i < n; ++i) {
            while (j < o.n && o.s[j] < s[i]) ++j;
            if (j == o.n || o.s[j] != s[i]) return false;
        }
        return true;
    }
};

struct DSU {
    std::vector<int64_t> p;
    explicit DSU(int64_t n) : p(n) { std::iota(p.begin(), p.end(), 0); }
    int64_t f(int64_t x) {
        while (p[x] != x) { p[x] = p[p[x]]; x = p[x]; }
        return x;
    }
    void u(int64_t a, int64_t b) {
        a = f(a); b = f(b);
        if (a != b) { if (a < b) p[b] = a; else p[a] = b; }
    }
};

bool sorted_strict_subset(const std::vector<int32_t> &a, const std::vector<int32_t> &b) {
    if (b.size() <= a.size()) return false;
    return std::includes(b.begin(), b.end(), a.begin(), a.end());
}

}  // namespace

int build_structure(const bddc_mesh *m, const bddc_partition *p, const double *coef,
                    const bddc_opts *o, Structure &st, std::string &err) {
    const int nx = m->nx, ny = m->ny, nz = m->nz;
    if (nx <= 0 || ny <= 0 || nz <= 0 || !(m->h > 0)) { err = "bad mesh size"; return BDDC_EINVAL; }
    const int64_t n1x = nx + 1, n1y = ny + 1;
    const int64_t nn = n1x * n1y * (nz + 1);
    const int64_t ne = (int64_t)nx * ny * nz;
    if (nn > INT32_MAX) { err = "mesh too large for int32 node ids"; return BDDC_EINVAL; }
    st.nx = nx; st.ny = ny; st.nz = nz; st.h = m->h; st.n_nodes = nn; st.n_elem = ne;
    const int nsub = p->n_sub;
    if (nsub <= 0 || !p->elem_to_sub || !coef) { err = "bad partition"; return BDDC_EINVAL; }
    auto kept = [&](int64_t e) { return m->elem_keep == nullptr || m->elem_keep[e] != 0; };
    auto enode = [&](int64_t e, int v) -> int64_t {
        int64_t ex = e % nx, ey = (e / nx) % ny, ez = e / ((int64_t)nx * ny);
        return (ex + (v & 1)) + n1x * ((ey + ((v >> 1) & 1)) + n1y * (ez + ((v >> 2) & 1)));
    };
    for (int64_t e = 0; e < ne; ++e) {
        if (!kept(e)) continue;
        if (p->elem_to_sub[e] < 0 || p->elem_to_sub[e] >= nsub) { err = "elem_to_sub out of range"; return BDDC_EINVAL; }
        if (!(coef[e] > 0) || !std::isfinite(coef[e])) { err = "coefficients must be positive and finite"; return BDDC_EINVAL; }
    }

    // S(n) for every node touched by a kept element
    std::vector<SubSet> S(nn);
    std::vector<double> csum(nn, 0.0);
    for (int64_t e = 0; e < ne; ++e) {
        if (!kept(e)) continue;
        for (int v = 0; v < 8; ++v) {
            int64_t n = enode(e, v);
            S[n].insert(p->elem_to_sub[e]);
            csum[n] += coef[e];
        }
    }
    std::vector<uint8_t> dir(nn, 0);
    for (int64_t n = 0; n < nn; ++n)
        dir[n] = m->node_dirichlet ? (m->node_dirichlet[n] != 0) : ((n % n1x) == nx);
    st.free_node.assign(nn, 0);
    for (int64_t n = 0; n < nn; ++n) st.free_node[n] = (S[n].n > 0 && !dir[n]);
    std::vector<int32_t> gidx(nn, -1);
    for (int64_t n = 0; n < nn; ++n)
        if (st.free_node[n] && S[n].n >= 2) { gidx[n] = (int32_t)st.gamma.size(); st.gamma.push_back((int32_t)n); }

    // globs: 6-connected components of nodes with |S| >= 2 and equal S
    DSU dsu(nn);
    auto nb_of = [&](int64_t n, int64_t *out) {
        int64_t ix = n % n1x, iy = (n / n1x) % n1y, iz = n / (n1x * n1y);
        int c = 0;
        if (ix > 0) out[c++] = n - 1;
        if (ix < nx) out[c++] = n + 1;
        if (iy > 0) out[c++] = n - n1x;
        if (iy < ny) out[c++] = n + n1x;
        if (iz > 0) out[c++] = n - n1x * n1y;
        if (iz < nz) out[c++] = n + n1x * n1y;
        return c;
    };
    for (int64_t n = 0; n < nn; ++n) {
        if (S[n].n < 2) continue;
        int64_t nb[6];
        int c = nb_of(n, nb);
        for (int t = 0; t < c; ++t)
            if (nb[t] > n && S[nb[t]].n >= 2 && S[nb[t]] == S[n]) dsu.u(n, nb[t]);
    }
    std::vector<int64_t> gsize(nn, 0);
    for (int64_t n = 0; n < nn; ++n)
        if (S[n].n >= 2) gsize[dsu.f(n)]++;

    // level-1 coarse DOFs
    std::vector<uint8_t> is_corner(nn, 0);
    if (o->constraints & BDDC_CORNERS) {
        for (int32_t n : st.gamma) {
            if (S[n].n < 3) continue;
            int64_t nb[6];
            int c = nb_of(n, nb);
            int64_t root = dsu.f(n);
            int in_glob = 0;
            bool superset = false;
            for (int t = 0; t < c; ++t) {
                if (S[nb[t]].n >= 2 && dsu.f(nb[t]) == root) ++in_glob;
                if (S[n].strict_subset_of(S[nb[t]])) superset = true;
            }
            if ((gsize[root] == 1 || in_glob <= 1) && !superset) {
                is_corner[n] = 1;
                CoarseDof d;
                d.kind = 0;
                d.nodes = {n};
                d.subs.assign(S[n].s, S[n].s + S[n].n);
                st.coarse.push_back(d);
                st.n_corner++;
            }
        }
    }
    {
        // globs in order of their smallest node id
        std::map<int64_t, std::vector<int64_t>> members;
        for (int64_t n = 0; n < nn; ++n)
            if (S[n].n >= 2) members[dsu.f(n)].push_back(n);
        for (int pass = 0; pass < 2; ++pass) {
            int want = pass == 0 ? BDDC_FACES : BDDC_EDGES;
            if (!(o->constraints & want)) continue;
            for (auto &kv : members) {
                const SubSet &s = S[kv.first];
                bool face = (s.n == 2);
                if ((pass == 0) != face) continue;
                CoarseDof d;
                d.kind = face ? 1 : 2;
                for (int64_t n : kv.second)
                    if (st.free_node[n] && !is_corner[n]) d.nodes.push_back(n);
                if (d.nodes.empty() || (!face && d.nodes.size() < 2)) continue;
                d.subs.assign(s.s, s.s + s.n);
                st.coarse.push_back(d);
                if (face) st.n_face++; else st.n_edge++;
            }
        }
    }
    const int nC = (int)st.coarse.size();

    // per-subdomain data
    st.n_sub = nsub;
    st.sub.assign(nsub, SubHost());
    for (int64_t e = 0; e < ne; ++e)
        if (kept(e)) st.sub[p->elem_to_sub[e]].elem.push_back((int32_t)e);
    std::vector<int32_t> pos(nn, -1);
    for (int i = 0; i < nsub; ++i) {
        SubHost &sh = st.sub[i];
        if (sh.elem.empty()) { err = "empty subdomain " + std::to_string(i); return BDDC_EINVAL; }
        std::vector<int32_t> loc;
        for (int32_t e : sh.elem)
            for (int v = 0; v < 8; ++v) {
                int64_t n = enode(e, v);
                if (st.free_node[n]) loc.push_back((int32_t)n);
            }
        std::sort(loc.begin(), loc.end());
        loc.erase(std::unique(loc.begin(), loc.end()), loc.end());
        for (int32_t n : loc) if (S[n].n == 1) sh.nodes.push_back(n);
        sh.nI = (int)sh.nodes.size();
        for (int32_t n : loc) if (S[n].n >= 2) sh.nodes.push_back(n);
        sh.nloc = (int)sh.nodes.size();
        sh.nB = sh.nloc - sh.nI;
        for (int k = 0; k < sh.nloc; ++k) pos[sh.nodes[k]] = k;
        sh.elem_loc.resize(sh.elem.size() * 8);
        sh.elem_c.resize(sh.elem.size());
        std::vector<int32_t> cnt(sh.nloc + 1, 0);
        for (size_t t = 0; t < sh.elem.size(); ++t) {
            int32_t e = sh.elem[t];
            sh.elem_c[t] = coef[e] * m->h;
            for (int v = 0; v < 8; ++v) {
                int64_t n = enode(e, v);
                int32_t l = st.free_node[n] ? pos[n] : -1;
                sh.elem_loc[t * 8 + v] = l;
                if (l >= 0) cnt[l + 1]++;
            }
        }
        sh.inc_ptr.assign(sh.nloc + 1, 0);
        for (int k = 0; k < sh.nloc; ++k) sh.inc_ptr[k + 1] = sh.inc_ptr[k] + cnt[k + 1];
        sh.inc_e.resize(sh.inc_ptr[sh.nloc]);
        sh.inc_v.resize(sh.inc_ptr[sh.nloc]);
        std::vector<int32_t> fill(sh.inc_ptr.begin(), sh.inc_ptr.end() - 1);
        for (size_t t = 0; t < sh.elem.size(); ++t)
            for (int v = 0; v < 8; ++v) {
                int32_t l = sh.elem_loc[t * 8 + v];
                if (l >= 0) { sh.inc_e[fill[l]] = (int32_t)t; sh.inc_v[fill[l]] = v; fill[l]++; }
            }
        // interface map and weights
        sh.gB.resize(sh.nB);
        sh.wB.resize(sh.nB);
        std::vector<double> own(sh.nB, 0.0);
        for (size_t t = 0; t < sh.elem.size(); ++t)
            for (int v = 0; v < 8; ++v) {
                int32_t l = sh.elem_loc[t * 8 + v];
                if (l >= sh.nI) own[l - sh.nI] += coef[sh.elem[t]];
            }
        for (int k = 0; k < sh.nB; ++k) {
            int32_t n = sh.nodes[sh.nI + k];
            sh.gB[k] = gidx[n];
            sh.wB[k] = (o->weights == 1) ? own[k] / csum[n] : 1.0 / S[n].n;
        }
        for (int32_t n : sh.nodes) pos[n] = -1;
    }
    (void)nC;
    int rc = constraint_rows(st, err);
    if (rc) return rc;
    return build_level2(st, p, err);
}


// Coarse DOFs of every subdomain (ascending) and its constraint rows over
// interface-local indices: the DOF's weights, or 1/|nodes| for an average
// (one node: a corner value).
int constraint_rows(Structure &st, std::string &err) {
    const int nC = (int)st.coarse.size();
    std::vector<int32_t> pos(st.n_nodes, -1);
    for (auto &sh : st.sub) {
        sh.cidx.clear();
        sh.c_ptr.clear();
        sh.c_col.clear();
        sh.c_val.clear();
    }
    for (int c = 0; c < nC; ++c)
        for (int32_t s : st.coarse[c].subs) st.sub[s].cidx.push_back(c);
    for (int i = 0; i < st.n_sub; ++i) {
        SubHost &sh = st.sub[i];
        for (int k = 0; k < sh.nB; ++k) pos[sh.nodes[sh.nI + k]] = k;
        sh.c_ptr.assign(1, 0);
        for (int32_t c : sh.cidx) {
            const CoarseDof &d = st.coarse[c];
            const double w = 1.0 / (double)d.nodes.size();
            for (size_t q = 0; q < d.nodes.size(); ++q) {
                const int64_t n = d.nodes[q];
                if (pos[n] < 0) { err = "coarse DOF outside its subdomain interface"; return BDDC_EINVAL; }
                sh.c_col.push_back(pos[n]);
                sh.c_val.push_back(d.wts.empty() ? w : d.wts[q]);
            }
            sh.c_ptr.push_back((int32_t)sh.c_col.size());
        }
        for (int k = 0; k < sh.nB; ++k) pos[sh.nodes[sh.nI + k]] = -1;
    }
    return BDDC_OK;
}

// Level-2 structure (three levels): subregion DOF lists, level-2 interface,
// globs, corners and face averages (the level-3 unknowns), constraint rows.
// Per subregion: its level-3 DOFs (ascending) and their rows over its
// level-2 interface positions (CSR).
static int level3_rows(Structure &st, std::string &err) {
    st.n3 = (int)st.dof3_members.size();
    std::vector<int32_t> posL(st.coarse.size(), -1);
    for (SubregionHost &r : st.sr) {
        r.c3.clear();
        r.c_ptr.clear();
        r.c_col.clear();
        r.c_val.clear();
    }
    for (int m3 = 0; m3 < st.n3; ++m3)
        for (int32_t j : st.dof3_subs[m3]) st.sr[j].c3.push_back(m3);
    for (SubregionHost &r : st.sr) {
        for (int k = 0; k < r.nB; ++k) posL[r.L[r.nI + k]] = k;
        r.c_ptr.assign(1, 0);
        for (int32_t m3 : r.c3) {
            const auto &mem = st.dof3_members[m3];
            const auto &w = st.dof3_wts[m3];
            for (size_t q = 0; q < mem.size(); ++q) {
                if (posL[mem[q]] < 0) { err = "level-2 constraint outside its subregion interface"; return BDDC_EINVAL; }
                r.c_col.push_back(posL[mem[q]]);
                r.c_val.push_back(w[q]);
            }
            r.c_ptr.push_back((int32_t)r.c_col.size());
        }
        for (int k = 0; k < r.nB; ++k) posL[r.L[r.nI + k]] = -1;
    }
    return BDDC_OK;
}

int build_level2(Structure &st, const bddc_partition *p, std::string &err) {
    const int nC = (int)st.coarse.size();
    const int nsub = st.n_sub;
    st.sr.clear();
    st.gamma2.clear();
    st.dof3_members.clear();
    st.dof3_subs.clear();
    st.dof3_wts.clear();
    st.dof3_kind.clear();
    st.n3 = st.n3_corner = st.n3_face = st.n3_adaptive = 0;
    st.three = p->n_subregion > 0;
    if (!st.three) return BDDC_OK;
    const int nsr = p->n_subregion;
    st.n_sr = nsr;
    if (!p->sub_to_subregion) { err = "sub_to_subregion missing"; return BDDC_EINVAL; }
    for (int i = 0; i < nsub; ++i)
        if (p->sub_to_subregion[i] < 0 || p->sub_to_subregion[i] >= nsr) { err = "sub_to_subregion out of range"; return BDDC_EINVAL; }
    std::vector<std::vector<int32_t>> S2(nC);
    for (int c = 0; c < nC; ++c) {
        for (int32_t s : st.coarse[c].subs) S2[c].push_back(p->sub_to_subregion[s]);
        std::sort(S2[c].begin(), S2[c].end());
        S2[c].erase(std::unique(S2[c].begin(), S2[c].end()), S2[c].end());
    }
    st.sr.assign(nsr, SubregionHost());
    for (int i = 0; i < nsub; ++i) st.sr[p->sub_to_subregion[i]].subs.push_back(i);
    std::vector<int32_t> g2idx(nC, -1);
    for (int c = 0; c < nC; ++c)
        if (S2[c].size() >= 2) { g2idx[c] = (int32_t)st.gamma2.size(); st.gamma2.push_back(c); }
    for (int j = 0; j < nsr; ++j) {
        SubregionHost &r = st.sr[j];
        if (r.subs.empty()) { err = "empty subregion " + std::to_string(j); return BDDC_EINVAL; }
        std::vector<int32_t> all;
        for (int32_t s : r.subs) all.insert(all.end(), st.sub[s].cidx.begin(), st.sub[s].cidx.end());
        std::sort(all.begin(), all.end());
        all.erase(std::unique(all.begin(), all.end()), all.end());
        for (int32_t c : all) if (S2[c].size() == 1) r.L.push_back(c);
        r.nI = (int)r.L.size();
        for (int32_t c : all) if (S2[c].size() >= 2) r.L.push_back(c);
        r.nB = (int)r.L.size() - r.nI;
        for (int k = 0; k < r.nB; ++k) {
            int32_t c = r.L[r.nI + k];
            r.g2.push_back(g2idx[c]);
            r.w.push_back(1.0 / (double)S2[c].size());
        }
    }
    // neighbour relation: coarse DOFs sharing a subdomain; level-2 globs
    DSU d2(nC);
    for (int i = 0; i < nsub; ++i) {
        const auto &ci = st.sub[i].cidx;
        for (size_t a = 0; a < ci.size(); ++a)
            for (size_t b = a + 1; b < ci.size(); ++b)
                if (g2idx[ci[a]] >= 0 && g2idx[ci[b]] >= 0 && S2[ci[a]] == S2[ci[b]] &&
                    st.coarse[ci[a]].kind != 3 && st.coarse[ci[b]].kind != 3)
                    d2.u(ci[a], ci[b]);
    }
    // adaptive face rows (Section 3.3) stay out of the level-2 globs: each one
    // on the level-2 interface is a level-3 unknown of its own, so the
    // operator does not depend on the rows' signs or on their basis
    std::map<int64_t, std::vector<int32_t>> gm;
    for (int32_t c : st.gamma2)
        if (st.coarse[c].kind != 3) gm[d2.f(c)].push_back(c);
    for (int32_t c : st.gamma2) {
        if (st.coarse[c].kind != 0 || S2[c].size() < 3) continue;
        std::vector<int32_t> nbs;
        for (int32_t s : st.coarse[c].subs) nbs.insert(nbs.end(), st.sub[s].cidx.begin(), st.sub[s].cidx.end());
        std::sort(nbs.begin(), nbs.end());
        nbs.erase(std::unique(nbs.begin(), nbs.end()), nbs.end());
        int64_t root = d2.f(c);
        int in_glob = 0;
        bool superset = false;
        for (int32_t mm : nbs) {
            if (mm == c) continue;
            if (g2idx[mm] >= 0 && d2.f(mm) == root) ++in_glob;
            if (sorted_strict_subset(S2[c], S2[mm])) superset = true;
        }
        if ((gm[root].size() == 1 || in_glob <= 1) && !superset) {
            st.dof3_members.push_back({c});
            st.dof3_subs.push_back(S2[c]);
            st.dof3_wts.push_back({1.0});
            st.dof3_kind.push_back(0);
            st.n3_corner++;
        }
    }
    for (int32_t c : st.gamma2) {
        if (st.coarse[c].kind != 3) continue;
        st.dof3_members.push_back({c});
        st.dof3_subs.push_back(S2[c]);
        st.dof3_wts.push_back({1.0});
        st.dof3_kind.push_back(3);
    }
    for (auto &kv : gm) {
        if (S2[kv.second[0]].size() != 2) continue;
        st.dof3_members.push_back(kv.second);
        st.dof3_subs.push_back(S2[kv.second[0]]);
        st.dof3_wts.push_back(std::vector<double>(kv.second.size(), 1.0 / (double)kv.second.size()));
        st.dof3_kind.push_back(1);
        st.n3_face++;
    }
    return level3_rows(st, err);
}

// Appends level-3 DOFs (adaptive rows of the level-2 faces) and rebuilds the
// subregions' constraint rows.
int add_level3_dofs(Structure &st, const std::vector<Level3Dof> &extra, std::string &err) {
    if (extra.empty()) return BDDC_OK;
    for (const Level3Dof &d : extra) {
        st.dof3_members.push_back(d.members);
        st.dof3_subs.push_back(d.subs);
        st.dof3_wts.push_back(d.wts);
        st.dof3_kind.push_back(4);
        st.n3_adaptive++;
    }
    return level3_rows(st, err);
}

// Appends coarse DOFs (adaptive face rows, Section 3.3) and rebuilds every
// subdomain's constraint rows and the level-2 structure.
int add_coarse_dofs(Structure &st, const bddc_partition *p, const std::vector<CoarseDof> &extra, std::string &err) {
    if (extra.empty()) return BDDC_OK;
    st.coarse.insert(st.coarse.end(), extra.begin(), extra.end());
    st.n_adaptive += (int)extra.size();
    int rc = constraint_rows(st, err);
    if (rc) return rc;
    return build_level2(st, p, err);
}

}  // namespace bddc
