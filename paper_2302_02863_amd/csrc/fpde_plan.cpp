// Host planning: rules, quadrature points, touching pairs, KD trees,
// admissibility and partitions, point location.  Compiled with
// -ffp-contract=off so that the structure-deciding arithmetic is reproducible.
#include "fpde_plan.h"
#include "fpde_threads.h"

#include <algorithm>
#include <cmath>
#include <numeric>
#include <stdexcept>

namespace fpde {

void gauss_legendre01(int n, double* x, double* w) {
    // Newton's method on P_n in binary128 arithmetic (113-bit mantissa), started
    // from the usual cosine estimate; rounding the converged value to double is
    // then correctly rounded for every n used by the rules.
    typedef __float128 q_t;
    auto qabs = [](q_t v) { return v < 0 ? -v : v; };
    auto legendre = [n](q_t t, q_t* pn, q_t* dpn) {
        q_t p0 = 1, p1 = t;
        for (int k = 2; k <= n; ++k) {
            q_t p2 = ((q_t)(2 * k - 1) * t * p1 - (q_t)(k - 1) * p0) / (q_t)k;
            p0 = p1;
            p1 = p2;
        }
        *pn = p1;
        *dpn = (n > 1) ? (q_t)n * (t * p1 - p0) / (t * t - 1) : (q_t)1;
    };
    std::vector<std::pair<q_t, q_t>> tw;
    const long double pi = 3.141592653589793238462643383279502884L;
    for (int i = 1; i <= n; ++i) {
        q_t t = (q_t)cosl(pi * ((long double)i - 0.25L) / ((long double)n + 0.5L));
        q_t pn, dp;
        for (int it = 0; it < 200; ++it) {
            legendre(t, &pn, &dp);
            q_t dt = pn / dp;
            t -= dt;
            if (qabs(dt) < (q_t)1e-30) break;
        }
        legendre(t, &pn, &dp);
        tw.push_back({t, (q_t)2 / ((1 - t * t) * dp * dp)});
    }
    std::sort(tw.begin(), tw.end(), [](const std::pair<q_t, q_t>& a, const std::pair<q_t, q_t>& b) {
        return a.first < b.first;
    });
    for (int i = 0; i < n; ++i) {
        double t = (double)tw[i].first;
        double ww = (double)tw[i].second;
        x[i] = 0.5 * (t + 1.0);
        w[i] = 0.5 * ww;
    }
}

ElementRule element_rule(int dim, int n) {
    ElementRule r;
    std::vector<double> g(n), w(n);
    gauss_legendre01(n, g.data(), w.data());
    if (dim == 1) {
        r.nqe = n;
        r.xh.assign(g.begin(), g.end());
        r.wh.assign(w.begin(), w.end());
        r.lam.resize(2 * n);
        for (int l = 0; l < n; ++l) {
            r.lam[l] = 1.0 - g[l];
            r.lam[n + l] = g[l];
        }
        return r;
    }
    r.nqe = n * n;
    r.xh.resize(2 * n * n);
    r.wh.resize(n * n);
    r.lam.resize(3 * n * n);
    for (int a = 0; a < n; ++a)
        for (int b = 0; b < n; ++b) {
            int l = a * n + b;
            double x0 = g[a], x1 = g[a] * g[b];
            r.xh[l] = x0;
            r.xh[n * n + l] = x1;
            r.wh[l] = (w[a] * w[b]) * g[a];
            r.lam[l] = 1.0 - x0;
            r.lam[n * n + l] = x0 - x1;
            r.lam[2 * n * n + l] = x1;
        }
    return r;
}

QuadPoints quad_points(const HostMesh& m, const ElementRule& r) {
    QuadPoints Q;
    Q.nqe = r.nqe;
    Q.nq = m.nc * r.nqe;
    Q.x.resize(m.dim * Q.nq);
    Q.w.resize(Q.nq);
    Q.q_int.resize(Q.nq);
    constexpr int64_t kChunk = 4096;   // cells per task; each cell writes its own points
    parallel_for((m.nc + kChunk - 1) / kChunk, [&](int64_t ch) {
        for (int64_t c = ch * kChunk; c < std::min(m.nc, (ch + 1) * kChunk); ++c) {
            if (m.dim == 1) {
                double v0 = m.x(0, m.v(0, c));
                double J = m.x(0, m.v(1, c)) - v0;
                double det = std::fabs(J);
                for (int l = 0; l < r.nqe; ++l) {
                    int64_t q = c * r.nqe + l;
                    Q.x[q] = v0 + J * r.xh[l];
                    Q.w[q] = det * r.wh[l];
                    Q.q_int[q] = m.interior[c];
                }
            } else {
                double J[2][2], v0[2];
                for (int d = 0; d < 2; ++d) {
                    v0[d] = m.x(d, m.v(0, c));
                    J[d][0] = m.x(d, m.v(1, c)) - m.x(d, m.v(0, c));
                    J[d][1] = m.x(d, m.v(2, c)) - m.x(d, m.v(1, c));
                }
                double det = std::fabs(J[0][0] * J[1][1] - J[0][1] * J[1][0]);
                for (int l = 0; l < r.nqe; ++l) {
                    int64_t q = c * r.nqe + l;
                    for (int d = 0; d < 2; ++d) {
                        double t = v0[d] + J[d][0] * r.xh[l];
                        Q.x[d * Q.nq + q] = t + J[d][1] * r.xh[r.nqe + l];
                    }
                    Q.w[q] = det * r.wh[l];
                    Q.q_int[q] = m.interior[c];
                }
            }
        }
    }, 2);
    return Q;
}

NodeCells node_cells(const HostMesh& m) {
    NodeCells nc;
    std::vector<int64_t> cnt(m.M + 1, 0);
    for (int64_t c = 0; c < m.nc; ++c)
        for (int a = 0; a <= m.dim; ++a) cnt[m.v(a, c) + 1]++;
    for (int64_t i = 0; i < m.M; ++i) cnt[i + 1] += cnt[i];
    nc.ptr = cnt;
    nc.cell.resize(cnt[m.M]);
    nc.slot.resize(cnt[m.M]);
    std::vector<int64_t> fill(cnt.begin(), cnt.end() - 1);
    for (int64_t c = 0; c < m.nc; ++c)
        for (int a = 0; a <= m.dim; ++a) {
            int64_t v = m.v(a, c);
            nc.cell[fill[v]] = c;
            nc.slot[fill[v]] = (int8_t)a;
            fill[v]++;
        }
    return nc;
}

std::vector<Pair> touching_pairs(const HostMesh& m, const NodeCells& ncs) {
    // chunks of cells on host threads, each chunk's pairs in cell order, then the
    // chunks concatenated in order: the same list as one pass over the cells
    constexpr int64_t kChunk = 4096;
    const int64_t nch = (m.nc + kChunk - 1) / kChunk;
    std::vector<std::vector<Pair>> part(nch);
    parallel_for(
        nch, [&](int64_t ch) { touching_pairs_range(m, ncs, ch * kChunk, std::min(m.nc, (ch + 1) * kChunk), part[ch]); },
        2);
    std::vector<Pair> out;
    size_t n = 0;
    for (auto& v : part) n += v.size();
    out.reserve(n);
    for (auto& v : part) out.insert(out.end(), v.begin(), v.end());
    return out;
}

void touching_pairs_range(const HostMesh& m, const NodeCells& ncs, int64_t cbeg, int64_t cend, std::vector<Pair>& out) {
    const int k = m.dim + 1;
    std::vector<int64_t> nbr;
    for (int64_t c = cbeg; c < cend; ++c) {
        int32_t vc[3];
        for (int a = 0; a < k; ++a) vc[a] = m.v(a, c);
        if (m.interior[c]) {
            Pair p{};
            p.kind = 0;
            p.c0 = p.c1 = (int32_t)c;
            int32_t s[3] = {vc[0], vc[1], k == 3 ? vc[2] : 0};
            std::sort(s, s + k);
            for (int a = 0; a < k; ++a) p.v[a] = p.v[3 + a] = s[a];
            out.push_back(p);
        }
        nbr.clear();
        for (int a = 0; a < k; ++a)
            for (int64_t e = ncs.ptr[vc[a]]; e < ncs.ptr[vc[a] + 1]; ++e)
                if (ncs.cell[e] > c) nbr.push_back(ncs.cell[e]);
        std::sort(nbr.begin(), nbr.end());
        nbr.erase(std::unique(nbr.begin(), nbr.end()), nbr.end());
        for (int64_t c2 : nbr) {
            if (!(m.interior[c] || m.interior[c2])) continue;
            int32_t v2[3];
            for (int a = 0; a < k; ++a) v2[a] = m.v(a, c2);
            std::vector<int32_t> sh;
            for (int a = 0; a < k; ++a)
                for (int b = 0; b < k; ++b)
                    if (vc[a] == v2[b]) sh.push_back(vc[a]);
            std::sort(sh.begin(), sh.end());
            Pair p{};
            p.c0 = (int32_t)c;
            p.c1 = (int32_t)c2;
            if ((int)sh.size() == k) throw std::runtime_error("duplicate cell");
            if (m.dim == 2 && sh.size() == 2) {
                p.kind = 1;
                int32_t t0 = -1, t1 = -1;
                for (int a = 0; a < 3; ++a) {
                    if (vc[a] != sh[0] && vc[a] != sh[1]) t0 = vc[a];
                    if (v2[a] != sh[0] && v2[a] != sh[1]) t1 = v2[a];
                }
                p.v[0] = sh[0]; p.v[1] = sh[1]; p.v[2] = t0;
                p.v[3] = sh[0]; p.v[4] = sh[1]; p.v[5] = t1;
            } else if (sh.size() == 1) {
                p.kind = 2;
                int32_t P = sh[0];
                std::vector<int32_t> o0, o1;
                for (int a = 0; a < k; ++a) {
                    if (vc[a] != P) o0.push_back(vc[a]);
                    if (v2[a] != P) o1.push_back(v2[a]);
                }
                std::sort(o0.begin(), o0.end());
                std::sort(o1.begin(), o1.end());
                p.v[0] = P; p.v[3] = P;
                for (size_t a = 0; a < o0.size(); ++a) {
                    p.v[1 + a] = o0[a];
                    p.v[4 + a] = o1[a];
                }
            } else {
                throw std::runtime_error("unexpected vertex sharing between cells");
            }
            out.push_back(p);
        }
    }
}

int pair_dofs(const HostMesh& m, const Pair& p, int32_t* o) {
    if (m.dim == 1) {
        if (p.kind == 0) { o[0] = p.v[0]; o[1] = p.v[1]; return 2; }
        o[0] = p.v[0]; o[1] = p.v[1]; o[2] = p.v[4]; return 3;
    }
    if (p.kind == 0) { o[0] = p.v[0]; o[1] = p.v[1]; o[2] = p.v[2]; return 3; }
    if (p.kind == 1) { o[0] = p.v[0]; o[1] = p.v[1]; o[2] = p.v[2]; o[3] = p.v[5]; return 4; }
    o[0] = p.v[0]; o[1] = p.v[1]; o[2] = p.v[2]; o[3] = p.v[4]; o[4] = p.v[5];
    return 5;
}

Tree kd_tree(int dim, const double* pts, int64_t stride, int64_t n, int leaf) {
    Tree t;
    t.dim = dim;
    t.n = n;
    int L = 0;
    while (((n + (int64_t(1) << L) - 1) >> L) > leaf) ++L;
    t.L = L;
    t.ncl = (int64_t(1) << (L + 1)) - 1;
    t.perm.resize(n);
    std::iota(t.perm.begin(), t.perm.end(), 0);
    t.beg.assign(t.ncl, 0);
    t.end.assign(t.ncl, 0);
    t.beg[0] = 0;
    t.end[0] = n;
    // level by level; the clusters of one level split disjoint ranges of perm
    auto split = [&](int64_t c) {
        int64_t b = t.beg[c], e = t.end[c];
        double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
        for (int64_t i = b; i < e; ++i)
            for (int k = 0; k < dim; ++k) {
                double v = pts[k * stride + t.perm[i]];
                lo[k] = std::min(lo[k], v);
                hi[k] = std::max(hi[k], v);
            }
        int axis = 0;
        for (int k = 1; k < dim; ++k)
            if (hi[k] - lo[k] > hi[axis] - lo[axis]) axis = k;
        const double* px = pts + axis * stride;
        const auto less = [px](int64_t i, int64_t j) {
            if (px[i] != px[j]) return px[i] < px[j];
            return i < j;
        };
        int64_t half = (e - b) / 2;
        // The split only needs the first half in (coordinate, id) order as a set; the last
        // internal level sorts fully, which fixes the order inside every leaf (and so the
        // whole permutation) exactly as full sorts at every level would.
        if (c >= (int64_t(1) << (L - 1)) - 1)
            std::sort(t.perm.begin() + b, t.perm.begin() + e, less);
        else
            std::nth_element(t.perm.begin() + b, t.perm.begin() + b + half, t.perm.begin() + e, less);
        t.beg[2 * c + 1] = b;
        t.end[2 * c + 1] = b + half;
        t.beg[2 * c + 2] = b + half;
        t.end[2 * c + 2] = e;
    };
    for (int lev = 0; lev < L; ++lev) {
        const int64_t c0 = (int64_t(1) << lev) - 1;
        parallel_for(int64_t(1) << lev, [&](int64_t i) { split(c0 + i); }, n >= 65536 ? 2 : 1 << 30);
    }
    return t;
}

void point_boxes(Tree& t, const double* pts, int64_t stride) {
    t.lo.assign(t.ncl * t.dim, 0.0);
    t.hi.assign(t.ncl * t.dim, 0.0);
    for (int64_t c = t.ncl - 1; c >= 0; --c) {
        for (int k = 0; k < t.dim; ++k) {
            double lo = 1e300, hi = -1e300;
            if (c >= t.first_leaf()) {
                for (int64_t i = t.beg[c]; i < t.end[c]; ++i) {
                    double v = pts[k * stride + t.perm[i]];
                    lo = std::min(lo, v);
                    hi = std::max(hi, v);
                }
            } else {
                lo = std::min(t.lo[(2 * c + 1) * t.dim + k], t.lo[(2 * c + 2) * t.dim + k]);
                hi = std::max(t.hi[(2 * c + 1) * t.dim + k], t.hi[(2 * c + 2) * t.dim + k]);
            }
            t.lo[c * t.dim + k] = lo;
            t.hi[c * t.dim + k] = hi;
        }
    }
}

bool admissible(int dim, const double* lo_a, const double* hi_a, const double* lo_b,
                const double* hi_b, double eta, double min_dist) {
    double s2 = 0.0;
    for (int k = 0; k < dim; ++k) {
        double dc = 0.5 * (lo_a[k] + hi_a[k]) - 0.5 * (lo_b[k] + hi_b[k]);
        s2 = s2 + dc * dc;
    }
    double dcent = std::sqrt(s2);
    double Da = 0.0, Db = 0.0, g2 = 0.0;
    for (int k = 0; k < dim; ++k) {
        double wa = hi_a[k] - lo_a[k];
        double wb = hi_b[k] - lo_b[k];
        Da = Da + wa * wa;
        Db = Db + wb * wb;
        double gap = std::max(0.0, std::max(lo_b[k] - hi_a[k], lo_a[k] - hi_b[k]));
        g2 = g2 + gap * gap;
    }
    Da = std::sqrt(Da);
    Db = std::sqrt(Db);
    return (eta * dcent >= 0.5 * (Da + Db)) && (std::sqrt(g2) > min_dist);
}

void sort_pairs(std::vector<std::pair<int64_t, int64_t>>& v, int64_t ncl) {
    const int64_t n = (int64_t)v.size();
    std::vector<int64_t> ptr(ncl + 1, 0), b(n);
    if (n < (int64_t(1) << 14)) {
        for (auto& x : v) ++ptr[x.first + 1];
        for (int64_t c = 0; c < ncl; ++c) ptr[c + 1] += ptr[c];
        std::vector<int64_t> fill(ptr.begin(), ptr.end() - 1);
        for (auto& x : v) b[fill[x.first]++] = x.second;
    } else {
        // counts and scatter on host threads with atomic counters: the order inside a
        // bucket then depends on the schedule, and the bucket sort below fixes it again
        constexpr int64_t kChunk = int64_t(1) << 16;
        const int64_t nch = (n + kChunk - 1) / kChunk;
        parallel_for(nch, [&](int64_t ch) {
            for (int64_t e = ch * kChunk; e < std::min(n, (ch + 1) * kChunk); ++e)
                __atomic_fetch_add(&ptr[v[e].first + 1], int64_t(1), __ATOMIC_RELAXED);
        }, 2);
        for (int64_t c = 0; c < ncl; ++c) ptr[c + 1] += ptr[c];
        std::vector<int64_t> fill(ptr.begin(), ptr.end() - 1);
        parallel_for(nch, [&](int64_t ch) {
            for (int64_t e = ch * kChunk; e < std::min(n, (ch + 1) * kChunk); ++e)
                b[__atomic_fetch_add(&fill[v[e].first], int64_t(1), __ATOMIC_RELAXED)] = v[e].second;
        }, 2);
    }
    parallel_for((ncl + 4095) / 4096, [&](int64_t blk) {
        const int64_t c1 = std::min(ncl, (blk + 1) * 4096);
        for (int64_t c = blk * 4096; c < c1; ++c) {
            std::sort(b.begin() + ptr[c], b.begin() + ptr[c + 1]);
            for (int64_t e = ptr[c]; e < ptr[c + 1]; ++e) v[e] = {c, b[e]};
        }
    });
}

void partition(const Tree& t, double eta, const std::vector<double>* hc, const std::vector<uint8_t>* skip,
               std::vector<std::pair<int64_t, int64_t>>& far,
               std::vector<std::pair<int64_t, int64_t>>& near) {
    far.clear();
    near.clear();
    const int d = t.dim;
    // one step of the dual-tree recursion: far, near (leaf pairs), or the four child pairs
    auto visit = [&](int64_t a, int64_t b, std::vector<std::pair<int64_t, int64_t>>& stack,
                     std::vector<std::pair<int64_t, int64_t>>& fo, std::vector<std::pair<int64_t, int64_t>>& no) {
        if (skip && (*skip)[a]) return;
        const double min_dist = hc ? (*hc)[a] + (*hc)[b] : 0.0;
        if (admissible(d, &t.lo[a * d], &t.hi[a * d], &t.lo[b * d], &t.hi[b * d], eta, min_dist)) {
            fo.push_back({a, b});
        } else if (a >= t.first_leaf()) {
            no.push_back({a, b});
        } else {
            for (int64_t ca : {2 * a + 1, 2 * a + 2})
                for (int64_t cb : {2 * b + 1, 2 * b + 2}) stack.push_back({ca, cb});
        }
    };
    // breadth first until there are enough independent subproblems, then each on its own
    std::vector<std::pair<int64_t, int64_t>> front{{0, 0}};
    while (!front.empty() && front.size() < 1024) {
        std::vector<std::pair<int64_t, int64_t>> next;
        for (auto& pr : front) visit(pr.first, pr.second, next, far, near);
        front.swap(next);
    }
    const int64_t nf = (int64_t)front.size();
    std::vector<std::vector<std::pair<int64_t, int64_t>>> fo(nf), no(nf);
    parallel_for(nf, [&](int64_t i) {
        std::vector<std::pair<int64_t, int64_t>> stack{front[i]};
        while (!stack.empty()) {
            auto pr = stack.back();
            stack.pop_back();
            visit(pr.first, pr.second, stack, fo[i], no[i]);
        }
    });
    for (int64_t i = 0; i < nf; ++i) {
        far.insert(far.end(), fo[i].begin(), fo[i].end());
        near.insert(near.end(), no[i].begin(), no[i].end());
    }
    sort_pairs(far, t.ncl);
    sort_pairs(near, t.ncl);
}

void cheb_axes(int dim, const double* lo, const double* hi, int p, double* out) {
    double D = 0.0;
    for (int k = 0; k < dim; ++k) D = D + (hi[k] - lo[k]) * (hi[k] - lo[k]);
    D = std::sqrt(D);
    const double pi = 3.14159265358979323846;
    for (int k = 0; k < dim; ++k) {
        double w = std::max(hi[k] - lo[k], 1e-12 * D);
        for (int a = 0; a < p; ++a) {
            double t = std::cos((2.0 * a + 1.0) * pi / (2.0 * p));
            out[k * p + a] = 0.5 * (lo[k] + hi[k]) + 0.5 * w * t;
        }
    }
}

std::vector<double> cell_diameters(const HostMesh& m) {
    std::vector<double> h(m.nc, 0.0);
    const int k = m.dim + 1;
    for (int64_t c = 0; c < m.nc; ++c)
        for (int a = 0; a < k; ++a)
            for (int b = a + 1; b < k; ++b) {
                double s = 0.0;
                for (int d = 0; d < m.dim; ++d) {
                    double dx = m.x(d, m.v(a, c)) - m.x(d, m.v(b, c));
                    s = s + dx * dx;
                }
                h[c] = std::max(h[c], std::sqrt(s));
            }
    return h;
}

std::vector<double> cluster_h(const Tree& t, const double* h_point) {
    std::vector<double> out(t.ncl, 0.0);
    for (int64_t c = t.ncl - 1; c >= 0; --c) {
        if (c >= t.first_leaf()) {
            for (int64_t i = t.beg[c]; i < t.end[c]; ++i) out[c] = std::max(out[c], h_point[t.perm[i]]);
        } else {
            out[c] = std::max(out[2 * c + 1], out[2 * c + 2]);
        }
    }
    return out;
}

// ------------------------------------------------------------------ locator

void Locator::build(const HostMesh& mesh) {
    m = &mesh;
    const int d = mesh.dim;
    double glo[2] = {1e300, 1e300}, ghi[2] = {-1e300, -1e300};
    for (int k = 0; k < d; ++k)
        for (int64_t v = 0; v < mesh.M; ++v) {
            glo[k] = std::min(glo[k], mesh.x(k, v));
            ghi[k] = std::max(ghi[k], mesh.x(k, v));
        }
    // bins about two mean cell widths wide (a graded mesh's few large cells go into
    // every bin they overlap)
    double vol = 1.0;
    for (int k = 0; k < d; ++k) vol *= std::max(ghi[k] - glo[k], 1e-300);
    double h = std::max(std::pow(vol / (double)std::max<int64_t>(mesh.nc, 1), 1.0 / d), 1e-300);
    for (int k = 0; k < 2; ++k) {
        if (k < d) {
            lo[k] = glo[k] - h;
            int64_t n = (int64_t)std::ceil((ghi[k] - glo[k] + 2 * h) / (2 * h)) + 1;
            nb[k] = std::max<int64_t>(1, std::min<int64_t>(n, 4096));
            inv[k] = nb[k] / (ghi[k] - glo[k] + 2 * h);
        } else {
            lo[k] = 0;
            nb[k] = 1;
            inv[k] = 0;
        }
    }
    auto bidx = [&](int k, double v) {
        int64_t b = (int64_t)std::floor((v - lo[k]) * inv[k]);
        return std::min<int64_t>(nb[k] - 1, std::max<int64_t>(0, b));
    };
    const int64_t NB = nb[0] * nb[1];
    std::vector<std::vector<int64_t>> bc(NB), bn(NB);
    for (int64_t c = 0; c < mesh.nc; ++c) {
        double clo[2] = {1e300, 1e300}, chi[2] = {-1e300, -1e300};
        for (int a = 0; a <= d; ++a)
            for (int k = 0; k < d; ++k) {
                clo[k] = std::min(clo[k], mesh.x(k, mesh.v(a, c)));
                chi[k] = std::max(chi[k], mesh.x(k, mesh.v(a, c)));
            }
        int64_t b0[2] = {0, 0}, b1[2] = {0, 0};
        for (int k = 0; k < d; ++k) {
            double pad = 1e-9 * h;
            b0[k] = bidx(k, clo[k] - pad);
            b1[k] = bidx(k, chi[k] + pad);
        }
        for (int64_t i = b0[0]; i <= b1[0]; ++i)
            for (int64_t j = b0[1]; j <= b1[1]; ++j) bc[i + nb[0] * j].push_back(c);
    }
    for (int64_t v = 0; v < mesh.M; ++v) {
        int64_t i = bidx(0, mesh.x(0, v));
        int64_t j = d > 1 ? bidx(1, mesh.x(1, v)) : 0;
        bn[i + nb[0] * j].push_back(v);
    }
    cptr.assign(NB + 1, 0);
    nptr.assign(NB + 1, 0);
    for (int64_t b = 0; b < NB; ++b) {
        cptr[b + 1] = cptr[b] + bc[b].size();
        nptr[b + 1] = nptr[b] + bn[b].size();
    }
    cells.reserve(cptr[NB]);
    nodes.reserve(nptr[NB]);
    for (int64_t b = 0; b < NB; ++b) {
        cells.insert(cells.end(), bc[b].begin(), bc[b].end());
        nodes.insert(nodes.end(), bn[b].begin(), bn[b].end());
    }
}

int64_t Locator::locate(const double* p, double* lam, int64_t* node) const {
    const HostMesh& mesh = *m;
    const int d = mesh.dim;
    auto bidx = [&](int k, double v) {
        int64_t b = (int64_t)std::floor((v - lo[k]) * inv[k]);
        return std::min<int64_t>(nb[k] - 1, std::max<int64_t>(0, b));
    };
    int64_t bi = bidx(0, p[0]);
    int64_t bj = d > 1 ? bidx(1, p[1]) : 0;
    int64_t b = bi + nb[0] * bj;
    const double tol = 1e-12;
    for (int64_t e = cptr[b]; e < cptr[b + 1]; ++e) {
        int64_t c = cells[e];
        if (d == 1) {
            double a = mesh.x(0, mesh.v(0, c)), bb = mesh.x(0, mesh.v(1, c));
            double t = (p[0] - a) / (bb - a);
            double L0 = 1.0 - t, L1 = t;
            if (L0 >= -tol && L1 >= -tol) {
                lam[0] = L0;
                lam[1] = L1;
                return c;
            }
        } else {
            double P0x = mesh.x(0, mesh.v(0, c)), P0y = mesh.x(1, mesh.v(0, c));
            double e1x = mesh.x(0, mesh.v(1, c)) - P0x, e1y = mesh.x(1, mesh.v(1, c)) - P0y;
            double e2x = mesh.x(0, mesh.v(2, c)) - P0x, e2y = mesh.x(1, mesh.v(2, c)) - P0y;
            double den = e1x * e2y - e1y * e2x;
            double dx = p[0] - P0x, dy = p[1] - P0y;
            double b1 = (dx * e2y - dy * e2x) / den;
            double b2 = (e1x * dy - e1y * dx) / den;
            double L0 = 1.0 - b1 - b2;
            if (L0 >= -tol && b1 >= -tol && b2 >= -tol) {
                lam[0] = L0;
                lam[1] = b1;
                lam[2] = b2;
                return c;
            }
        }
    }
    // nearest node: ring search over node buckets
    double best = 1e300;
    int64_t bestv = -1;
    double bw[2] = {1.0 / inv[0], d > 1 ? 1.0 / inv[1] : 0.0};
    for (int64_t r = 0;; ++r) {
        bool any = false;
        for (int64_t i = bi - r; i <= bi + r; ++i) {
            for (int64_t j = (d > 1 ? bj - r : 0); j <= (d > 1 ? bj + r : 0); ++j) {
                bool ring = (std::llabs(i - bi) == r) || (d > 1 && std::llabs(j - bj) == r);
                if (!ring) continue;
                if (i < 0 || i >= nb[0] || j < 0 || j >= nb[1]) continue;
                any = true;
                int64_t bb = i + nb[0] * j;
                for (int64_t e = nptr[bb]; e < nptr[bb + 1]; ++e) {
                    int64_t v = nodes[e];
                    double s = 0.0;
                    for (int k = 0; k < d; ++k) {
                        double dd = mesh.x(k, v) - p[k];
                        s = s + dd * dd;
                    }
                    if (s < best || (s == best && v < bestv)) {
                        best = s;
                        bestv = v;
                    }
                }
            }
        }
        double minw = d > 1 ? std::min(bw[0], bw[1]) : bw[0];
        double lb = (r) * minw;   // every node in ring r+1 or beyond is at least this far
        if (bestv >= 0 && lb * lb > best) break;
        if (!any && r > nb[0] + nb[1] + 2) break;
    }
    *node = bestv;
    return -1;
}

}  // namespace fpde
