// Host-side FP64 mathematics of the engine: bond Hamiltonians of the
// XYZ-plus-fields chain, gate exponentials G_b = exp(-i (T/2) h_b) (Sec. III A,
// Eq. (5)), their parameter derivatives for the reverse-mode gradient, dense
// fused window matrices, and the product-state factor tables.
//
// The exponential of a 4x4 Hermitian h is taken through its eigendecomposition
// h = V diag(lambda) V^dagger, computed with the cyclic complex Jacobi method
// (Jacobi 1846; e.g. Golub & Van Loan, "Matrix Computations", Sec. 8.5):
// exp(-i tau h) = V diag(exp(-i tau lambda)) V^dagger.  Derivatives use the
// Daleckii-Krein formula: for f = exp and X = -i tau h = V diag(x) V^dagger,
//   Df(X)[E] = V (Gamma o (V^dagger E V)) V^dagger,
//   Gamma_kl = (e^{x_k} - e^{x_l}) / (x_k - x_l)
//            = e^{-i tau (l_k + l_l)/2} sinc(tau (l_k - l_l)/2),
// which stays exact for (near-)degenerate eigenvalues.
#include "host_math.h"

#include <cmath>
#include <cstdint>
#include <cstring>

namespace fl {

using cd = std::complex<double>;

static void mat4_mul(const cd* A, const cd* B, cd* C) {
    cd t[16];
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            cd s = 0;
            for (int k = 0; k < 4; ++k) s += A[4 * i + k] * B[4 * k + j];
            t[4 * i + j] = s;
        }
    std::memcpy(C, t, sizeof(t));
}

static void mat4_adj(const cd* A, cd* B) {
    cd t[16];
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) t[4 * i + j] = std::conj(A[4 * j + i]);
    std::memcpy(B, t, sizeof(t));
}

void herm_eig4(const cd* h, double* lam, cd* V) {
    cd A[16];
    for (int i = 0; i < 16; ++i) A[i] = h[i];
    // symmetrise: A = (h + h^dagger)/2 so that rounding in the input cannot
    // leave a non-Hermitian residue
    for (int i = 0; i < 4; ++i)
        for (int j = i; j < 4; ++j) {
            cd s = 0.5 * (A[4 * i + j] + std::conj(A[4 * j + i]));
            A[4 * i + j] = s;
            A[4 * j + i] = std::conj(s);
        }
    for (int i = 0; i < 16; ++i) V[i] = (i % 5 == 0) ? cd(1.0) : cd(0.0);
    for (int sweep = 0; sweep < 64; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int i = 0; i < 4; ++i)
            for (int j = 0; j < 4; ++j) {
                double a = std::norm(A[4 * i + j]);
                tot += a;
                if (i != j) off += a;
            }
        if (off <= 1e-34 * tot || off == 0.0) break;
        for (int p = 0; p < 3; ++p)
            for (int q = p + 1; q < 4; ++q) {
                const cd apq = A[4 * p + q];
                const double r = std::abs(apq);
                if (r == 0.0) continue;
                // phase that makes the (p,q) entry real and positive
                const cd ph = apq / r;
                const double app = A[4 * p + p].real(), aqq = A[4 * q + q].real();
                // real Jacobi rotation zeroing the real symmetric 2x2 block
                const double zeta = (aqq - app) / (2.0 * r);
                const double t = (zeta >= 0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
                const double c = 1.0 / std::sqrt(1.0 + t * t);
                const double s = t * c;
                // U = D R with D = diag(1,..,conj(ph) at q,..), R the rotation
                // U[p][p] = c, U[p][q] = s, U[q][p] = -s conj(ph), U[q][q] = c conj(ph)
                cd U[16];
                for (int i = 0; i < 16; ++i) U[i] = (i % 5 == 0) ? cd(1.0) : cd(0.0);
                U[4 * p + p] = c;
                U[4 * p + q] = s;
                U[4 * q + p] = -s * std::conj(ph);
                U[4 * q + q] = c * std::conj(ph);
                cd Ud[16];
                mat4_adj(U, Ud);
                mat4_mul(Ud, A, A);
                mat4_mul(A, U, A);
                mat4_mul(V, U, V);
                A[4 * p + q] = 0.0;
                A[4 * q + p] = 0.0;
            }
    }
    for (int i = 0; i < 4; ++i) lam[i] = A[4 * i + i].real();
}

void gate_exp(const cd* h, double tau, cd* G) {
    double lam[4];
    cd V[16];
    herm_eig4(h, lam, V);
    cd D[16];
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) D[4 * i + j] = V[4 * i + j] * std::polar(1.0, -tau * lam[j]);
    cd Vd[16];
    mat4_adj(V, Vd);
    mat4_mul(D, Vd, G);
    // one Newton-Schulz step towards the unitary polar factor:
    // G <- G (3 I - G^dagger G) / 2 (removes the O(eps) non-unitarity)
    cd Gd[16], GG[16];
    mat4_adj(G, Gd);
    mat4_mul(Gd, G, GG);
    for (int i = 0; i < 16; ++i) GG[i] = ((i % 5 == 0) ? cd(3.0) : cd(0.0)) - GG[i];
    mat4_mul(G, GG, G);
    for (int i = 0; i < 16; ++i) G[i] *= 0.5;
}

static cd sinc_phase(double tau, double lk, double ll) {
    const double y = 0.5 * tau * (lk - ll);
    const double sc = (std::fabs(y) < 1e-8) ? 1.0 - y * y / 6.0 : std::sin(y) / y;
    return std::polar(sc, -0.5 * tau * (lk + ll));
}

void gate_exp_derivative(const cd* h, const cd* gen, double tau, cd* dG) {
    double lam[4];
    cd V[16];
    herm_eig4(h, lam, V);
    cd Vd[16], E[16], T[16];
    mat4_adj(V, Vd);
    // E = V^dagger (-i tau gen) V
    for (int i = 0; i < 16; ++i) T[i] = cd(0.0, -tau) * gen[i];
    mat4_mul(Vd, T, E);
    mat4_mul(E, V, E);
    for (int k = 0; k < 4; ++k)
        for (int l = 0; l < 4; ++l) E[4 * k + l] *= sinc_phase(tau, lam[k], lam[l]);
    mat4_mul(V, E, E);
    mat4_mul(E, Vd, dG);
}

void xyz_bond(const double* J3, const double* fl3, const double* fr3, cd* h) {
    // Pauli matrices, local index 2*bit_left + bit_right; left factor acts on
    // the lower site of the bond.
    const cd X[4] = {0, 1, 1, 0};
    const cd Y[4] = {0, cd(0, -1), cd(0, 1), 0};
    const cd Z[4] = {1, 0, 0, -1};
    const cd I[4] = {1, 0, 0, 1};
    const cd* P[3] = {X, Y, Z};
    for (int i = 0; i < 16; ++i) h[i] = 0.0;
    auto kron_add = [&](const cd* A, const cd* B, cd w) {
        for (int a0 = 0; a0 < 2; ++a0)
            for (int b0 = 0; b0 < 2; ++b0)
                for (int a1 = 0; a1 < 2; ++a1)
                    for (int b1 = 0; b1 < 2; ++b1)
                        h[4 * (2 * a0 + b0) + (2 * a1 + b1)] += w * A[2 * a0 + a1] * B[2 * b0 + b1];
    };
    for (int a = 0; a < 3; ++a) {
        kron_add(P[a], P[a], J3[a]);
        kron_add(P[a], I, 0.5 * fl3[a]);
        kron_add(I, P[a], 0.5 * fr3[a]);
    }
}

void mat_mul_n(const cd* A, const cd* B, cd* C, int n) {
    std::vector<cd> t((size_t)n * n);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            cd s = 0;
            for (int k = 0; k < n; ++k) s += A[(size_t)i * n + k] * B[(size_t)k * n + j];
            t[(size_t)i * n + j] = s;
        }
    std::memcpy(C, t.data(), sizeof(cd) * n * n);
}

void embed_gate(const cd* G, int nbits, int i, cd* U) {
    // U = I (x) G (x) I acting on window bits (i, i+1) of an nbits-bit window;
    // window index w, local gate index 2*bit(i+1) + bit(i).
    const int n = 1 << nbits;
    for (int r = 0; r < n * n; ++r) U[r] = 0.0;
    for (int w = 0; w < n; ++w) {
        const int rest = w & ~(3 << i);
        const int col_l = (w >> i) & 3;
        for (int row_l = 0; row_l < 4; ++row_l) {
            const int wr = rest | (row_l << i);
            U[(size_t)wr * n + w] += G[4 * row_l + col_l];
        }
    }
}

void window_matrix_bits(const cd* const* gates, const int* pos, int nops, int nbits, cd* U) {
    const int n = 1 << nbits;
    std::vector<cd> E((size_t)n * n);
    for (int r = 0; r < n * n; ++r) U[r] = (r % (n + 1) == 0) ? cd(1.0) : cd(0.0);
    for (int k = 0; k < nops; ++k) {
        embed_gate(gates[k], nbits, pos[k], E.data());
        mat_mul_n(E.data(), U, U, n);
    }
}

void window_matrix(const cd* const* gates, const int* pos, int nops, cd* U) {
    window_matrix_bits(gates, pos, nops, 6, U);
}

// 4-bit window index with bits (i, i+1) = the local index a (bit i = a & 1)
// and the other two bits = z, in order.
static inline int ins2(int a, int z, int i) {
    const int lo = z & ((1 << i) - 1);
    const int hi = z >> i;
    return lo | (a << i) | (hi << (i + 2));
}

void window_overlap_terms(const cd* Q, const cd* const* gates, const int* pos, int nops, double* out) {
    // T = the 16x16 window overlap sum psi_x conj(lambda_y) before op k; the
    // op's gate G (local index 2 bit(i+1) + bit(i)) then maps T to G T G^dagger.
    cd T[256], U[256];
    for (int e = 0; e < 256; ++e) T[e] = Q[e];
    for (int k = 0; k < nops; ++k) {
        const int i = pos[k];
        // R[a][b] = sum over the other two window bits of T
        cd R[16];
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b) {
                cd s = 0.0;
                for (int z = 0; z < 4; ++z) s += T[ins2(a, z, i) * 16 + ins2(b, z, i)];
                R[4 * a + b] = s;
            }
        // sum conj(lambda_l) psi_m - conj(psi_l) lambda_m = R[m][l] - conj(R[l][m]);
        // the diagonal keeps Im R[l][l] (half of the purely imaginary entry)
        double* o = out + (size_t)k * 16;
        for (int l = 0; l < 4; ++l) o[l] = R[5 * l].imag();
        int q = 4;
        for (int l = 0; l < 4; ++l)
            for (int m = l + 1; m < 4; ++m) {
                const cd d = R[4 * m + l] - std::conj(R[4 * l + m]);
                o[q] = d.real();
                o[q + 1] = d.imag();
                q += 2;
            }
        // T <- G T G^dagger on window bits (i, i+1)
        const cd* G = gates[k];
        for (int z = 0; z < 4; ++z)
            for (int y = 0; y < 16; ++y)
                for (int a = 0; a < 4; ++a) {
                    cd s = 0.0;
                    for (int a2 = 0; a2 < 4; ++a2) s += G[4 * a + a2] * T[ins2(a2, z, i) * 16 + y];
                    U[ins2(a, z, i) * 16 + y] = s;
                }
        for (int x = 0; x < 16; ++x)
            for (int z = 0; z < 4; ++z)
                for (int b = 0; b < 4; ++b) {
                    cd s = 0.0;
                    for (int b2 = 0; b2 < 4; ++b2) s += U[x * 16 + ins2(b2, z, i)] * std::conj(G[4 * b + b2]);
                    T[x * 16 + ins2(b, z, i)] = s;
                }
    }
}

void window_fragments4(const cd* U, float* out) {
    // real form A[2m'+c'][2m+c] of the 16x16 complex U with its columns taken
    // component-major, k' = 16 c + m: lane l, step s holds A[l % 32][k] for
    // k' = 2 s + l / 32, i.e. m = k' mod 16, c = k' / 16, so that steps s and
    // s + 8 take the real and imaginary part of one amplitude
    for (int l = 0; l < 64; ++l)
        for (int st = 0; st < 16; ++st) {
            const int r = l & 31, kc = 2 * st + (l >> 5);
            const int k = 2 * (kc & 15) + (kc >> 4);
            const cd u = U[(r >> 1) * 16 + (k >> 1)];
            double a;
            if ((r & 1) == 0) a = (k & 1) == 0 ? u.real() : -u.imag();
            else a = (k & 1) == 0 ? u.imag() : u.real();
            out[l * 16 + st] = (float)a;
        }
}

double bf16_rne(double a) {
    if (a == 0.0 || !std::isfinite(a)) return a;
    int e = 0;
    std::frexp(a, &e);                        // a = f 2^e, 0.5 <= |f| < 1
    const double scale = std::ldexp(1.0, e - 8);   // 8 significant bits
    return std::nearbyint(a / scale) * scale;      // ties to even (default rounding mode)
}

static uint16_t bf16_bits(double v) {
    const float f = (float)v;  // exact: v has at most 8 significant bits
    uint32_t u;
    std::memcpy(&u, &f, 4);
    return (uint16_t)(u >> 16);
}

void window_fragments(const cd* U, int mode, void* out) {
    auto A = [&](int r, int k) -> double {
        const int mr = r >> 1, cr = r & 1, mk = k >> 1, ck = k & 1;
        const cd u = U[mr * 64 + mk];
        if (cr == 0) return ck == 0 ? u.real() : -u.imag();
        return ck == 0 ? u.imag() : u.real();
    };
    if (mode == 0) {
        float* o = static_cast<float*>(out);
        for (int w = 0; w < 4; ++w)
            for (int l = 0; l < 64; ++l)
                for (int kk = 0; kk < 64; ++kk)
                    o[(w * 64 + l) * 64 + kk] = (float)A(32 * w + (l & 31), 2 * kk + (l >> 5));
    } else {
        // Rows 2m' and 2m'+1 of the real form hold the same numbers, (Re, -Im)
        // and (Im, Re) of U[m'][m] at columns (2m, 2m+1); store each (Re, Im)
        // pair once, split hi/lo, and let the kernel negate or swap per row.
        // Chunk ((w * 8 + st) * 2 + lk) * 16 + mm holds, for m' = 16 w + mm,
        // the pairs of m = 8 st + 4 lk .. + 3 (8 bf16); hi plane, then lo.
        uint16_t* hi = static_cast<uint16_t*>(out);
        uint16_t* lo = hi + 8192;
        for (int w = 0; w < 4; ++w)
            for (int st = 0; st < 8; ++st)
                for (int lk = 0; lk < 2; ++lk)
                    for (int mm = 0; mm < 16; ++mm)
                        for (int j = 0; j < 4; ++j) {
                            const cd u = U[(16 * w + mm) * 64 + 8 * st + 4 * lk + j];
                            const size_t idx = ((size_t)((w * 8 + st) * 2 + lk) * 16 + mm) * 8 + 2 * j;
                            const double parts[2] = {u.real(), u.imag()};
                            for (int c = 0; c < 2; ++c) {
                                const double h = bf16_rne(parts[c]);
                                hi[idx + c] = bf16_bits(h);
                                lo[idx + c] = bf16_bits(bf16_rne(parts[c] - h));
                            }
                        }
    }
}

void product_tables(int L, const cd* spinors, int a, int b, std::vector<cd>& tlo,
                    std::vector<cd>& tmid, std::vector<cd>& thi) {
    // x = (xhi << (a+b)) | (xmid << a) | xlo; bit q of x belongs to site L-1-q.
    auto build = [&](int first_bit, int nbits, std::vector<cd>& t) {
        t.assign((size_t)1 << nbits, cd(1.0));
        for (int v = 0; v < (1 << nbits); ++v) {
            cd p = 1.0;
            for (int k = 0; k < nbits; ++k) {
                const int q = first_bit + k;
                const int site = L - 1 - q;
                p *= spinors[2 * site + ((v >> k) & 1)];
            }
            t[v] = p;
        }
    };
    build(0, a, tlo);
    build(a, b, tmid);
    build(a + b, L - a - b, thi);
}

void ground_state4(const cd* h, cd* g, double* e0) {
    double lam[4];
    cd V[16];
    herm_eig4(h, lam, V);
    int j = 0;
    for (int k = 1; k < 4; ++k)
        if (lam[k] < lam[j]) j = k;
    int big = 0;
    for (int i = 1; i < 4; ++i)
        if (std::abs(V[4 * i + j]) > std::abs(V[4 * big + j])) big = i;
    const cd ph = std::conj(V[4 * big + j]) / std::abs(V[4 * big + j]);
    double nrm = 0.0;
    for (int i = 0; i < 4; ++i) nrm += std::norm(V[4 * i + j]);
    nrm = std::sqrt(nrm);
    for (int i = 0; i < 4; ++i) g[i] = V[4 * i + j] * ph / nrm;
    if (e0) *e0 = lam[j];
}

bool pair_tables(int L, const cd* pairs, const cd* tail, int a, int b, std::vector<cd>& tlo,
                 std::vector<cd>& tmid, std::vector<cd>& thi) {
    // bit q of x belongs to site L-1-q; pair m holds sites (2m, 2m+1), i.e.
    // bits qa = L-1-2m (the high bit of its local index) and qb = qa-1
    const int npairs = L / 2;
    auto build = [&](int q0, int n, std::vector<cd>& t) -> bool {
        t.assign((size_t)1 << n, cd(1.0));
        for (int m = 0; m < npairs; ++m) {
            const int qa = L - 1 - 2 * m, qb = qa - 1;
            const bool ia = qa >= q0 && qa < q0 + n, ib = qb >= q0 && qb < q0 + n;
            if (ia != ib) return false;   // a boundary would split the pair
            if (!ia) continue;
            for (int v = 0; v < (1 << n); ++v) {
                const int loc = 2 * ((v >> (qa - q0)) & 1) + ((v >> (qb - q0)) & 1);
                t[v] *= pairs[4 * m + loc];
            }
        }
        if ((L & 1) && q0 == 0 && n > 0)   // the unpaired last site is bit 0
            for (int v = 0; v < (1 << n); ++v) t[v] *= tail[v & 1];
        return true;
    };
    return build(0, a, tlo) && build(a, b, tmid) && build(a + b, L - a - b, thi);
}

}  // namespace fl
