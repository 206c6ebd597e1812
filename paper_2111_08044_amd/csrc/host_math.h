// Host-side FP64 mathematics (see host_math.cpp).
#pragma once
#include <complex>
#include <vector>

namespace fl {

// Eigendecomposition of a 4x4 Hermitian matrix (row-major): h = V diag(lam) V^dagger.
void herm_eig4(const std::complex<double>* h, double* lam, std::complex<double>* V);

// G = exp(-i tau h) for a 4x4 Hermitian h.
void gate_exp(const std::complex<double>* h, double tau, std::complex<double>* G);

// d/dtheta exp(-i tau h(theta)) in the direction dh/dtheta = gen.
void gate_exp_derivative(const std::complex<double>* h, const std::complex<double>* gen,
                         double tau, std::complex<double>* dG);

// Bond Hamiltonian Jx XX + Jy YY + Jz ZZ + (1/2) fl.sigma (x) I + (1/2) I (x) fr.sigma.
void xyz_bond(const double* J3, const double* fl3, const double* fr3, std::complex<double>* h);

// C = A B for n x n row-major complex matrices (C may alias A or B).
void mat_mul_n(const std::complex<double>* A, const std::complex<double>* B,
               std::complex<double>* C, int n);

// Embed a 4x4 gate on bits (i, i+1) of an nbits-bit window into a 2^nbits matrix.
void embed_gate(const std::complex<double>* G, int nbits, int i, std::complex<double>* U);

// U = E(op_{n-1}) ... E(op_0) on an nbits-bit window, E = gate gates[k]
// embedded at window bits (pos[k], pos[k]+1).  U: 2^nbits x 2^nbits row-major.
void window_matrix_bits(const std::complex<double>* const* gates, const int* pos, int nops, int nbits,
                        std::complex<double>* U);
// The 6-bit case (U: 64x64).
void window_matrix(const std::complex<double>* const* gates, const int* pos, int nops, std::complex<double>* U);

// Overlap terms of the ops of one 4-bit register group of the reverse pass,
// from the group's window overlap Q[x][y] = sum_r psi_{r,x} conj(lambda_{r,y})
// (16x16 complex, row-major) taken before its first op.  Op k applies
// gates[k] (4x4, local index 2 bit(pos+1) + bit(pos)) on window bits
// (pos[k], pos[k]+1); out[k][16] receives its bond's terms at the state before
// the gate, in the reverse kernel's layout: [0..3] Im(conj(lambda_l) psi_l),
// then (re, im) of sum conj(lambda_l) psi_m - conj(psi_l) lambda_m for the
// pairs 01, 02, 03, 12, 13, 23.
void window_overlap_terms(const std::complex<double>* Q, const std::complex<double>* const* gates, const int* pos,
                          int nops, double* out);

// MFMA fragments of the real 32x32 form of a 16x16 complex window matrix
// (k = 2m + (0 re, 1 im)): out[lane * 16 + s] = A[lane % 32][2 s + lane / 32],
// 1024 floats (4 KiB).
void window_fragments4(const std::complex<double>* U, float* out);

// Round-to-nearest-even to bfloat16 (8 significant bits), returned as a double.
double bf16_rne(double a);

// Per-lane MFMA fragments of the real 128x128 form of a 64x64 complex window
// matrix (rows/columns ordered k = 2m + (0 re, 1 im)).  mode 0: 16384 floats
// (64 KiB), [wave][lane][kk] = A[32 wave + lane%32][2 kk + lane/32].  mode 1:
// the (Re, Im) pairs of U, each stored once (rows 2m' and 2m'+1 of A hold the
// same numbers), 8192 uint16 bf16 hi then 8192 lo (32 KiB):
// [wave][step][lk][mm][j][c] = part c of U[16 wave + mm][8 step + 4 lk + j];
// a lane with row 32 wave + lane%32 = 2m' + c' takes its 8 values
// A[2m'+c'][16 step + 8 lk + i] as (Re, -Im) pairs for c' = 0, (Im, Re) for 1.
void window_fragments(const std::complex<double>* U, int mode, void* out);

// Factor tables of a product state psi[x] = thi[x >> (a+b)] tmid[(x >> a) & (2^b-1)] tlo[x & (2^a-1)].
void product_tables(int L, const std::complex<double>* spinors, int a, int b,
                    std::vector<std::complex<double>>& tlo, std::vector<std::complex<double>>& tmid,
                    std::vector<std::complex<double>>& thi);

// Lowest eigenvector of a 4x4 Hermitian h (unit norm, largest component real
// and positive); *e0 (if not NULL) receives its eigenvalue.
void ground_state4(const std::complex<double>* h, std::complex<double>* g, double* e0);

// Factor tables (as product_tables) of the pair-product state
// psi[x] = prod_m pairs[m][2 bit(site 2m) + bit(site 2m+1)] (* tail[bit(site L-1)]
// for odd L).  false if a table boundary (a or a+b) would split a pair.
bool pair_tables(int L, const std::complex<double>* pairs, const std::complex<double>* tail, int a, int b,
                 std::vector<std::complex<double>>& tlo, std::vector<std::complex<double>>& tmid,
                 std::vector<std::complex<double>>& thi);

}  // namespace fl
