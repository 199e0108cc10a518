// jw.cpp -- the qubit Hamiltonian of Eq. (3) (arXiv 2601.09951, Section 3.2)
// by a symbolic Jordan-Wigner map, on the host.
//
// Pauli strings are kept in symplectic form P(x, z) = i^{|x&z|} X^x Z^z over
// amplitude-index bits (wire w = bit n-1-w).  Products follow from
// Z^a X^b = (-1)^{|a&b|} X^b Z^a:
//   P(x1,z1) P(x2,z2) = i^{|x1&z1| + |x2&z2| - |x&z| + 2|z1&x2|} P(x1^x2, z1^z2).
// Mode P (wire P) carries a_P = Z_{<P} (X_P + i Y_P)/2 and
// a+_P = Z_{<P} (X_P - i Y_P)/2 with |1> = occupied, i.e. in this form
//   a_P  = 1/2 P(b, zs) + i/2 P(b, zs|b),   a+_P = 1/2 P(b, zs) - i/2 P(b, zs|b)
// with b the bit of wire P and zs the bits of wires 0..P-1.
#include <algorithm>
#include <cmath>
#include <complex>
#include <numeric>
#include <unordered_map>

#include "internal.h"

namespace vqe {

namespace {

using cd = std::complex<double>;

struct PStr {
    uint64_t x, z;
    cd c;
};

inline int popc(uint64_t v) { return __builtin_popcountll(v); }

inline cd ipow(int e)
{
    switch (e & 3) {
    case 0: return {1, 0};
    case 1: return {0, 1};
    case 2: return {-1, 0};
    default: return {0, -1};
    }
}

inline PStr mul(const PStr &a, const PStr &b)
{
    uint64_t x = a.x ^ b.x, z = a.z ^ b.z;
    int e = popc(a.x & a.z) + popc(b.x & b.z) - popc(x & z) + 2 * popc(a.z & b.x);
    return {x, z, a.c * b.c * ipow(((e % 4) + 4) % 4)};
}

// the two-string expansion of a_P (dag = false) or a+_P (dag = true)
inline void ladder(int n, int P, bool dag, PStr out[2])
{
    uint64_t b = 1ull << (n - 1 - P);
    uint64_t zs = 0;
    for (int Q = 0; Q < P; ++Q) zs |= 1ull << (n - 1 - Q);
    out[0] = {b, zs, cd(0.5, 0)};
    out[1] = {b, zs | b, cd(0, dag ? -0.5 : 0.5)};
}

struct KeyHash {
    size_t operator()(const std::pair<uint64_t, uint64_t> &k) const
    {
        return std::hash<uint64_t>()(k.first * 0x9E3779B97F4A7C15ull ^ k.second);
    }
};

}  // namespace

void merge_terms(std::vector<uint64_t> &x, std::vector<uint64_t> &z, std::vector<double> &c,
                 double drop)
{
    std::vector<size_t> order(x.size());
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) {
        return x[a] != x[b] ? x[a] < x[b] : z[a] < z[b];
    });
    std::vector<uint64_t> X, Z;
    std::vector<double> C;
    for (size_t i = 0; i < order.size();) {
        size_t j = i;
        double s = 0;
        while (j < order.size() && x[order[j]] == x[order[i]] && z[order[j]] == z[order[i]]) {
            s += c[order[j]];
            ++j;
        }
        if (std::fabs(s) > drop) {
            X.push_back(x[order[i]]);
            Z.push_back(z[order[i]]);
            C.push_back(s);
        }
        i = j;
    }
    x.swap(X);
    z.swap(Z);
    c.swap(C);
}

int jordan_wigner(int n_orb, const double *h1, const double *h2, double e_core,
                  std::vector<uint64_t> &xo, std::vector<uint64_t> &zo, std::vector<double> &co,
                  std::string &err)
{
    const int M = 2 * n_orb;
    const int n = M;
    std::unordered_map<std::pair<uint64_t, uint64_t>, cd, KeyHash> acc;
    auto add = [&](const PStr &s) { acc[{s.x, s.z}] += s.c; };

    for (int i = 0; i < n_orb * n_orb; ++i)
        if (!std::isfinite(h1[i])) { err = "non-finite one-electron integral"; return VQE_EINVAL; }
    const size_t n2 = (size_t)n_orb * n_orb * n_orb * n_orb;
    for (size_t i = 0; i < n2; ++i)
        if (!std::isfinite(h2[i])) { err = "non-finite two-electron integral"; return VQE_EINVAL; }
    if (!std::isfinite(e_core)) { err = "non-finite core energy"; return VQE_EINVAL; }

    if (e_core != 0.0) add({0, 0, cd(e_core, 0)});

    PStr lp[2], lq[2], lr[2], ls[2];
    // one-body part: sum_{PQ} h_PQ a+_P a_Q, spin conserved
    for (int P = 0; P < M; ++P) {
        ladder(n, P, true, lp);
        for (int Q = 0; Q < M; ++Q) {
            if ((P & 1) != (Q & 1)) continue;
            double h = h1[(P / 2) * n_orb + (Q / 2)];
            if (h == 0.0) continue;
            ladder(n, Q, false, lq);
            for (auto &a : lp)
                for (auto &b : lq) {
                    PStr s = mul(a, b);
                    s.c *= h;
                    add(s);
                }
        }
    }
    // two-body part: 1/2 sum_{PQRS} (p s|q r) a+_P a+_Q a_R a_S, spin of P = S, Q = R
    auto g = [&](int p, int q, int r, int s) {
        return h2[(((size_t)p * n_orb + q) * n_orb + r) * n_orb + s];
    };
    for (int P = 0; P < M; ++P) {
        ladder(n, P, true, lp);
        for (int Q = 0; Q < M; ++Q) {
            if (Q == P) continue;
            ladder(n, Q, true, lq);
            PStr pq[4];
            for (int a = 0; a < 2; ++a)
                for (int b = 0; b < 2; ++b) pq[2 * a + b] = mul(lp[a], lq[b]);
            for (int R = 0; R < M; ++R) {
                if ((R & 1) != (Q & 1)) continue;
                ladder(n, R, false, lr);
                for (int S = 0; S < M; ++S) {
                    if (S == R || (S & 1) != (P & 1)) continue;
                    double v = g(P / 2, S / 2, Q / 2, R / 2);
                    if (v == 0.0) continue;
                    ladder(n, S, false, ls);
                    for (auto &ab : pq)
                        for (auto &c3 : lr) {
                            PStr t = mul(ab, c3);
                            for (auto &d : ls) {
                                PStr u = mul(t, d);
                                u.c *= 0.5 * v;
                                add(u);
                            }
                        }
                }
            }
        }
    }
    xo.clear();
    zo.clear();
    co.clear();
    for (auto &kv : acc) {
        const cd c = kv.second;
        if (std::abs(c) <= 1e-14) continue;
        if (std::fabs(c.imag()) > 1e-12 * std::max(1.0, std::fabs(c.real()))) {
            err = "Jordan-Wigner image has a complex coefficient: integrals lack the required symmetry";
            return VQE_EINVAL;
        }
        xo.push_back(kv.first.first);
        zo.push_back(kv.first.second);
        co.push_back(c.real());
    }
    merge_terms(xo, zo, co, 1e-14);
    return VQE_OK;
}

// The same expansion with the integrals kept symbolic: every Pauli string's
// coefficient is a linear form in the integral entries.  Entries are
// numbered in the input layout {e_core, h1[n][n], h2[n][n][n][n]}, and every
// entry is mapped to the first entry of its symmetry class (h1 symmetric,
// h2 with the 8-fold permutational symmetry), so the imaginary parts of the
// weights cancel and the map is real for symmetric integrals.
int jordan_wigner_linear(int n_orb, std::vector<uint64_t> &xo, std::vector<uint64_t> &zo,
                         std::vector<int64_t> &row_off, std::vector<int32_t> &col,
                         std::vector<double> &val, std::string &err)
{
    const int M = 2 * n_orb;
    const int n = M;
    const int64_t n1 = (int64_t)n_orb * n_orb;
    auto h1_index = [&](int p, int q) {
        if (q < p) std::swap(p, q);
        return (int32_t)(1 + (int64_t)p * n_orb + q);
    };
    auto h2_index = [&](int p, int q, int r, int s) {
        int cand[8][4] = {{p, q, r, s}, {q, p, r, s}, {p, q, s, r}, {q, p, s, r},
                          {r, s, p, q}, {s, r, p, q}, {r, s, q, p}, {s, r, q, p}};
        int64_t best = -1;
        for (auto &c : cand) {
            int64_t v = (((int64_t)c[0] * n_orb + c[1]) * n_orb + c[2]) * n_orb + c[3];
            if (best < 0 || v < best) best = v;
        }
        return (int32_t)(1 + n1 + best);
    };
    std::unordered_map<std::pair<uint64_t, uint64_t>, std::unordered_map<int32_t, cd>, KeyHash> acc;
    auto add = [&](const PStr &s, int32_t e, double scale) { acc[{s.x, s.z}][e] += s.c * scale; };
    add({0, 0, cd(1, 0)}, 0, 1.0);

    PStr lp[2], lq[2], lr[2], ls[2];
    for (int P = 0; P < M; ++P) {
        ladder(n, P, true, lp);
        for (int Q = 0; Q < M; ++Q) {
            if ((P & 1) != (Q & 1)) continue;
            ladder(n, Q, false, lq);
            const int32_t e = h1_index(P / 2, Q / 2);
            for (auto &a : lp)
                for (auto &b : lq) add(mul(a, b), e, 1.0);
        }
    }
    for (int P = 0; P < M; ++P) {
        ladder(n, P, true, lp);
        for (int Q = 0; Q < M; ++Q) {
            if (Q == P) continue;
            ladder(n, Q, true, lq);
            PStr pq[4];
            for (int a = 0; a < 2; ++a)
                for (int b = 0; b < 2; ++b) pq[2 * a + b] = mul(lp[a], lq[b]);
            for (int R = 0; R < M; ++R) {
                if ((R & 1) != (Q & 1)) continue;
                ladder(n, R, false, lr);
                for (int S = 0; S < M; ++S) {
                    if (S == R || (S & 1) != (P & 1)) continue;
                    ladder(n, S, false, ls);
                    const int32_t e = h2_index(P / 2, S / 2, Q / 2, R / 2);
                    for (auto &ab : pq)
                        for (auto &c3 : lr) {
                            PStr t = mul(ab, c3);
                            for (auto &d : ls) add(mul(t, d), e, 0.5);
                        }
                }
            }
        }
    }
    // deterministic order: strings by (x, z), entries ascending
    std::vector<std::pair<uint64_t, uint64_t>> keys;
    for (auto &kv : acc) keys.push_back(kv.first);
    std::sort(keys.begin(), keys.end());
    xo.clear();
    zo.clear();
    row_off.assign(1, 0);
    col.clear();
    val.clear();
    for (auto &k : keys) {
        std::vector<std::pair<int32_t, double>> row;
        for (auto &ev : acc[k]) {
            const cd w = ev.second;
            if (std::fabs(w.imag()) > 1e-12) {
                err = "internal error: non-real symbolic Jordan-Wigner weight";
                return VQE_EINVAL;
            }
            if (std::fabs(w.real()) > 1e-14) row.push_back({ev.first, w.real()});
        }
        if (row.empty()) continue;
        std::sort(row.begin(), row.end());
        xo.push_back(k.first);
        zo.push_back(k.second);
        for (auto &r : row) {
            col.push_back(r.first);
            val.push_back(r.second);
        }
        row_off.push_back((int64_t)col.size());
    }
    return VQE_OK;
}

}  // namespace vqe
