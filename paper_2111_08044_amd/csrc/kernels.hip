// HIP kernels of the Floquet brickwork engine (gfx950, wave64).
//
//  k_sweep_tiles / k_sweep
//             fused gate sweep: one HBM read + write of the state applies
//             every gate of a pass (Sec. II Eq. (2), fused as in Sec. II).
//  k_rdm_groups / k_rdm_tiles / k_rdm
//             two-site reduced density matrices of the bonds of a pass (plus
//             the norm): exact products of the stored amplitudes, FP64 sums
//             (Sec. II Eq. (1); Sec. IV Eq. (10)).
//  k_apply_h  lambda = H0 psi, out of place (Sec. IV Eq. (11), Sec. V).
//  k_adjoint  reverse replay with G^dagger and the overlap terms of the
//             gradient of <H0>.
//  k_dense6 / k_dense4
//             pre-multiplied 6-qubit (FP32 or split BF16x3) and 4-qubit (FP32)
//             windows on the matrix cores (Sec. II on half-precision matrix
//             units).
//  k_init     product initial state (Sec. IV Eq. (9) form; product of spinors).
//  k_overlap  <phi|psi> and both norms across precisions (Sec. V echo measure).
//  k_finalize deterministic sum of per-workgroup partials.
//
// Tile kernels hold a tile of 2^K amplitudes (see fl_common.h for the
// geometry); each thread keeps 2^R amplitudes of one register group in VGPRs,
// applies the group's 4x4 gates there, and the tile changes register layout
// between groups through LDS.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "fl_common.h"
#include "kernels.h"

namespace fl {

template <typename T> struct CT;
template <> struct CT<float> { typedef float2 c; };
template <> struct CT<double> { typedef double2 c; };

typedef float fl_f32x4 __attribute__((ext_vector_type(4)));
typedef float fl_f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 fl_bf16x8 __attribute__((ext_vector_type(8)));

// ---------------------------------------------------------------------------
// register-level gate application
// ---------------------------------------------------------------------------

// out_i = sum_j G_ij a_j on the four amplitudes whose register index has bits
// (I, I+1) = local index (2*bit(I+1) + bit(I)), for every value of the other
// R-2 register bits.  G holds 16 complex entries, row-major, (re, im) pairs.
template <typename T, int R, int I>
__device__ __forceinline__ void apply_pair(T (&vr)[1 << R], T (&vi)[1 << R], const T* __restrict__ G) {
    __asm__ volatile("; gate on register bits %0" ::"i"(I));
    T g[32];
#pragma unroll
    for (int k = 0; k < 32; ++k) g[k] = G[k];
#pragma unroll
    for (int c = 0; c < (1 << (R - 2)); ++c) {
        const int b = (c & ((1 << I) - 1)) | ((c >> I) << (I + 2));
        T ar[4], ai[4];
#pragma unroll
        for (int l = 0; l < 4; ++l) {
            ar[l] = vr[b | (l << I)];
            ai[l] = vi[b | (l << I)];
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            T sr = g[8 * i] * ar[0];
            T si = g[8 * i] * ai[0];
            sr = fma(-g[8 * i + 1], ai[0], sr);
            si = fma(g[8 * i + 1], ar[0], si);
#pragma unroll
            for (int j = 1; j < 4; ++j) {
                sr = fma(g[8 * i + 2 * j], ar[j], sr);
                sr = fma(-g[8 * i + 2 * j + 1], ai[j], sr);
                si = fma(g[8 * i + 2 * j], ai[j], si);
                si = fma(g[8 * i + 2 * j + 1], ar[j], si);
            }
            vr[b | (i << I)] = sr;
            vi[b | (i << I)] = si;
        }
    }
    __asm__ volatile("; end gate on register bits %0" ::"i"(I));
}

// Same, with the 16 complex gate entries already in registers (SGPRs: the
// gate is uniform across the workgroup), updating the amplitudes in place.
// Every output first sums the seven terms that do not hold its own input
// amplitude; the last FMA of output (re|im)_i then adds the diagonal term
// Re(G_ii) (re|im)_i.  That FMA is the last read of its input, so it can
// write the result into the input's own register: each variant ends with
// every amplitude in the register it started in, and the variants for
// different I rejoin without register copies.
// The empty asm markers carry the bit position as an immediate: they keep the
// optimizer from merging the variants for different I into one body with
// run-time register indices (which would force the arrays into scratch).
template <typename T, int R, int I>
__device__ __forceinline__ void apply_pair_g(T (&vr)[1 << R], T (&vi)[1 << R], const T (&g)[32]) {
    __asm__ volatile("; gate on register bits %0" ::"i"(I));
#pragma unroll
    for (int c = 0; c < (1 << (R - 2)); ++c) {
        const int b = (c & ((1 << I) - 1)) | ((c >> I) << (I + 2));
        T sr[4], si[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int e = b | (i << I);
            sr[i] = -g[8 * i + 2 * i + 1] * vi[e];
            si[i] = g[8 * i + 2 * i + 1] * vr[e];
#pragma unroll
            for (int jj = 1; jj < 4; ++jj) {
                const int j = (i + jj) & 3;
                const int f = b | (j << I);
                sr[i] = fma(g[8 * i + 2 * j], vr[f], sr[i]);
                sr[i] = fma(-g[8 * i + 2 * j + 1], vi[f], sr[i]);
                si[i] = fma(g[8 * i + 2 * j], vi[f], si[i]);
                si[i] = fma(g[8 * i + 2 * j + 1], vr[f], si[i]);
            }
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int e = b | (i << I);
            vr[e] = fma(g[8 * i + 2 * i], vr[e], sr[i]);
            vi[e] = fma(g[8 * i + 2 * i], vi[e], si[i]);
        }
    }
    __asm__ volatile("; end gate on register bits %0" ::"i"(I));
}

// Calls f(std::integral_constant<int, I>) for the run-time bit position
// i in [0, R-2].  The last position is the switch default, so every path of
// the switch applies a gate: a path that did nothing would rejoin the others
// with the untouched values and cost register copies at the join.
template <int R, typename F>
__device__ __forceinline__ void with_bit(int i, F&& f) {
    static_assert(R >= 2 && R <= 5, "register group size");
    if constexpr (R == 2) {
        f(std::integral_constant<int, 0>{});
    } else if constexpr (R == 3) {
        switch (i) {
            case 0: f(std::integral_constant<int, 0>{}); break;
            default: f(std::integral_constant<int, 1>{}); break;
        }
    } else if constexpr (R == 4) {
        switch (i) {
            case 0: f(std::integral_constant<int, 0>{}); break;
            case 1: f(std::integral_constant<int, 1>{}); break;
            default: f(std::integral_constant<int, 2>{}); break;
        }
    } else {
        switch (i) {
            case 0: f(std::integral_constant<int, 0>{}); break;
            case 1: f(std::integral_constant<int, 1>{}); break;
            case 2: f(std::integral_constant<int, 2>{}); break;
            default: f(std::integral_constant<int, 3>{}); break;
        }
    }
}

template <typename T, int R>
__device__ __forceinline__ void apply_op_g(T (&vr)[1 << R], T (&vi)[1 << R], int i, const T (&g)[32]) {
    with_bit<R>(i, [&](auto I) { apply_pair_g<T, R, decltype(I)::value>(vr, vi, g); });
}

// Out-of-place form: reads every amplitude of (sr, si) and writes the result
// to (dr, di).  All variants write the same destination registers, so the
// run-time choice of I needs no register moves where the variants rejoin.
template <typename T, int R, int I>
__device__ __forceinline__ void apply_pair_to(const T (&sr)[1 << R], const T (&si)[1 << R], T (&dr)[1 << R],
                                              T (&di)[1 << R], const T (&g)[32]) {
    __asm__ volatile("; gate on register bits %0 (out of place)" ::"i"(I));
#pragma unroll
    for (int c = 0; c < (1 << (R - 2)); ++c) {
        const int b = (c & ((1 << I) - 1)) | ((c >> I) << (I + 2));
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            T ar = g[8 * i] * sr[b];
            T ai = g[8 * i] * si[b];
            ar = fma(-g[8 * i + 1], si[b], ar);
            ai = fma(g[8 * i + 1], sr[b], ai);
#pragma unroll
            for (int j = 1; j < 4; ++j) {
                ar = fma(g[8 * i + 2 * j], sr[b | (j << I)], ar);
                ar = fma(-g[8 * i + 2 * j + 1], si[b | (j << I)], ar);
                ai = fma(g[8 * i + 2 * j], si[b | (j << I)], ai);
                ai = fma(g[8 * i + 2 * j + 1], sr[b | (j << I)], ai);
            }
            dr[b | (i << I)] = ar;
            di[b | (i << I)] = ai;
        }
    }
    __asm__ volatile("; end gate on register bits %0 (out of place)" ::"i"(I));
}

template <typename T, int R>
__device__ __forceinline__ void apply_op_to(const T (&sr)[1 << R], const T (&si)[1 << R], T (&dr)[1 << R],
                                            T (&di)[1 << R], int i, const T (&g)[32]) {
    if constexpr (R >= 2) if (i == 0) { apply_pair_to<T, R, 0>(sr, si, dr, di, g); return; }
    if constexpr (R >= 3) if (i == 1) { apply_pair_to<T, R, 1>(sr, si, dr, di, g); return; }
    if constexpr (R >= 4) if (i == 2) { apply_pair_to<T, R, 2>(sr, si, dr, di, g); return; }
    if constexpr (R >= 5) if (i == 3) { apply_pair_to<T, R, 3>(sr, si, dr, di, g); return; }
}

template <typename T, int R>
__device__ __forceinline__ void apply_op(T (&vr)[1 << R], T (&vi)[1 << R], int i, const T* __restrict__ G) {
    if constexpr (R >= 2) if (i == 0) { apply_pair<T, R, 0>(vr, vi, G); return; }
    if constexpr (R >= 3) if (i == 1) { apply_pair<T, R, 1>(vr, vi, G); return; }
    if constexpr (R >= 4) if (i == 2) { apply_pair<T, R, 2>(vr, vi, G); return; }
    if constexpr (R >= 5) if (i == 3) { apply_pair<T, R, 3>(vr, vi, G); return; }
}

// ---------------------------------------------------------------------------
// tile load / store (global <-> LDS), 16-byte global accesses
// ---------------------------------------------------------------------------

// LDS slot of tile element j: fl_swz (SW = 0) or fl_swz12 (SW = 1)
template <int SW>
__device__ __forceinline__ uint32_t tile_swz(uint32_t j) {
    return SW ? fl_swz12(j) : fl_swz(j);
}

template <typename T, int KT, int NT = FL_NT, int SW = 0>
__device__ __forceinline__ void tile_load(const typename CT<T>::c* __restrict__ psi, uint64_t base, int K, int C,
                                          int h, typename CT<T>::c* lds) {
    typedef typename CT<T>::c cplx;
    if constexpr (sizeof(T) == 4) {
        const int n2 = 1 << (K - 1);  // pairs of amplitudes
        if constexpr (KT > 0) {
            constexpr int ITER = (1 << (KT - 1)) / NT;
            float4 v[ITER];
#pragma unroll
            for (int s = 0; s < ITER; ++s) {
                const uint32_t j = 2u * (threadIdx.x + s * NT);
                // streaming: each amplitude is read once per pass
                const fl_f32x4 t =
                    __builtin_nontemporal_load(reinterpret_cast<const fl_f32x4*>(psi + base + fl_tile_offset(j, C, h)));
                v[s] = make_float4(t[0], t[1], t[2], t[3]);
            }
#pragma unroll
            for (int s = 0; s < ITER; ++s) {
                const uint32_t j = 2u * (threadIdx.x + s * NT);
                lds[tile_swz<SW>(j)] = make_float2(v[s].x, v[s].y);
                lds[tile_swz<SW>(j + 1)] = make_float2(v[s].z, v[s].w);
            }
        } else {
            for (int p = threadIdx.x; p < n2; p += NT) {
                const uint32_t j = 2u * p;
                const float4 v = *reinterpret_cast<const float4*>(psi + base + fl_tile_offset(j, C, h));
                lds[tile_swz<SW>(j)] = make_float2(v.x, v.y);
                lds[tile_swz<SW>(j + 1)] = make_float2(v.z, v.w);
            }
        }
    } else {
        const int n = 1 << K;
        if constexpr (KT > 0) {
            constexpr int ITER = (1 << KT) / NT;
            cplx v[ITER];
#pragma unroll
            for (int s = 0; s < ITER; ++s) {
                const uint32_t j = threadIdx.x + s * NT;
                v[s] = psi[base + fl_tile_offset(j, C, h)];
            }
#pragma unroll
            for (int s = 0; s < ITER; ++s) lds[tile_swz<SW>(threadIdx.x + s * NT)] = v[s];
        } else {
            for (int j = threadIdx.x; j < n; j += NT) lds[tile_swz<SW>(j)] = psi[base + fl_tile_offset(j, C, h)];
        }
    }
}

template <typename T, int KT, int NT = FL_NT, int SW = 0>
__device__ __forceinline__ void tile_store(typename CT<T>::c* __restrict__ psi, uint64_t base, int K, int C, int h,
                                           const typename CT<T>::c* lds) {
    if constexpr (sizeof(T) == 4) {
        const int n2 = 1 << (K - 1);
        if constexpr (KT > 0) {
            constexpr int ITER = (1 << (KT - 1)) / NT;
#pragma unroll
            for (int s = 0; s < ITER; ++s) {
                const uint32_t j = 2u * (threadIdx.x + s * NT);
                const float2 a = lds[tile_swz<SW>(j)], b = lds[tile_swz<SW>(j + 1)];
                const fl_f32x4 t = {a.x, a.y, b.x, b.y};
                __builtin_nontemporal_store(t, reinterpret_cast<fl_f32x4*>(psi + base + fl_tile_offset(j, C, h)));
            }
        } else {
            for (int p = threadIdx.x; p < n2; p += NT) {
                const uint32_t j = 2u * p;
                const float2 a = lds[tile_swz<SW>(j)], b = lds[tile_swz<SW>(j + 1)];
                *reinterpret_cast<float4*>(psi + base + fl_tile_offset(j, C, h)) = make_float4(a.x, a.y, b.x, b.y);
            }
        }
    } else {
        const int n = 1 << K;
        for (int j = threadIdx.x; j < n; j += NT) psi[base + fl_tile_offset(j, C, h)] = lds[tile_swz<SW>(j)];
    }
}

// ---------------------------------------------------------------------------
// fused sweep
// ---------------------------------------------------------------------------

template <typename T, int R, int KT, int KMAX>
__global__ __launch_bounds__(FL_NT) void k_sweep(typename CT<T>::c* __restrict__ psi, const T* __restrict__ gates,
                                                 int C, int W, fl_pass pd) {
    typedef typename CT<T>::c cplx;
    __shared__ cplx lds[1 << KMAX];
    const int K = KT > 0 ? KT : C + W;
    const int h = pd.h;
    const uint64_t base = fl_tile_base(blockIdx.x, C, W, h);
    tile_load<T, KT>(psi, base, K, C, h, lds);
    __syncthreads();
    const uint32_t nsub = 1u << (K - R);
    for (int g = 0; g < pd.ngroups; ++g) {
        const int u0 = pd.u0[g];
        const int nops = pd.nops[g];
        for (uint32_t o = threadIdx.x; o < nsub; o += FL_NT) {
            const uint32_t b0 = fl_spread(o, u0, R);
            T vr[1 << R], vi[1 << R];
#pragma unroll
            for (int m = 0; m < (1 << R); ++m) {
                const cplx a = lds[fl_swz(b0 | ((uint32_t)m << u0))];
                vr[m] = a.x;
                vi[m] = a.y;
            }
            for (int q = 0; q < nops; ++q) {
                const int gi = pd.opg[g][q];
                if (gi >= 0) apply_op<T, R>(vr, vi, pd.opi[g][q], gates + 32 * gi);
            }
#pragma unroll
            for (int m = 0; m < (1 << R); ++m) {
                cplx a;
                a.x = vr[m];
                a.y = vi[m];
                lds[fl_swz(b0 | ((uint32_t)m << u0))] = a;
            }
        }
        __syncthreads();
    }
    tile_store<T, KT>(psi, base, K, C, h, lds);
}

// Op q of group g as (gate-table index, register bit), read as aligned 32-bit
// words of the pass descriptor so that the loads stay scalar (sub-dword
// loads of the kernel arguments would go through the vector memory path).
typedef int32_t __attribute__((may_alias)) fl_i32a;
__device__ __forceinline__ int pass_gate(const fl_pass& pd, int g, int q) {
    const int32_t w = reinterpret_cast<const fl_i32a*>(&pd.opg[g][0])[q >> 1];
    return (q & 1) ? (w >> 16) : (int)(int16_t)(w & 0xffff);
}
__device__ __forceinline__ int pass_slot(const fl_pass& pd, int g, int q) {
    const int32_t w = reinterpret_cast<const fl_i32a*>(&pd.ops[g][0])[q >> 1];
    return (q & 1) ? (w >> 16) : (int)(int16_t)(w & 0xffff);
}
__device__ __forceinline__ int pass_byte(const int8_t* row, int i) {
    const int32_t w = reinterpret_cast<const fl_i32a*>(row)[i >> 2];
    return (int)(int8_t)((w >> (8 * (i & 3))) & 0xff);
}
__device__ __forceinline__ int pass_u0(const fl_pass& pd, int g) { return pass_byte(pd.u0, g); }
__device__ __forceinline__ int pass_nops(const fl_pass& pd, int g) { return pass_byte(pd.nops, g); }
__device__ __forceinline__ int pass_bit(const fl_pass& pd, int g, int q) {
    const int32_t w = reinterpret_cast<const fl_i32a*>(&pd.opi[g][0])[q >> 2];
    return (w >> (8 * (q & 3))) & 0xff;
}

// lgkmcnt(0) with no wait on the vector-memory and export counters.
#define FL_WAIT_LGKM0 0xc07f

// The ops of register group g applied to the SUB register groups of a
// thread.  Ops run two per iteration (the register copies that LLVM places on
// a loop back edge after the 4-way choice of gate bits are then not needed at
// all).  The next op's gate (32 scalar registers) is fetched while the
// current one is applied; an explicit lgkmcnt(0) before each fetch waits for
// the previous one, so that no wait inside an apply ever covers the fetch in
// flight.  gc holds the group's first gate on entry and the next group's
// first gate on return: that fetch overlaps the LDS exchange between the two
// groups instead of stalling the start of the next group.
template <typename T, int R, int SUB>
__device__ __forceinline__ void sweep_group_ops(T (&vr)[SUB][1 << R], T (&vi)[SUB][1 << R], const fl_pass& pd, int g,
                                                const T* __restrict__ gates, T (&gc)[32]) {
    const int nops = pass_nops(pd, g);
    const int ng = pd.ngroups;
    auto gate_of = [&](int q) {
        const int idx = q < nops ? pass_gate(pd, g, q) : (g + 1 < ng ? pass_gate(pd, g + 1, 0) : pass_gate(pd, g, nops - 1));
        return gates + 32 * idx;
    };
    int i = pass_bit(pd, g, 0);
    T g1[32];
    for (int q = 0; q < nops; q += 2) {
        __builtin_amdgcn_s_waitcnt(FL_WAIT_LGKM0);
        const int i1 = pass_bit(pd, g, q + 1 < nops ? q + 1 : q);
        {
            const T* G = gate_of(q + 1);
#pragma unroll
            for (int k = 0; k < 32; ++k) g1[k] = G[k];
        }
#pragma unroll
        for (int s = 0; s < SUB; ++s) apply_op_g<T, R>(vr[s], vi[s], i, gc);
        if (q + 1 < nops) {
            __builtin_amdgcn_s_waitcnt(FL_WAIT_LGKM0);
            i = pass_bit(pd, g, q + 2 < nops ? q + 2 : q + 1);
            {
                const T* G = gate_of(q + 2);
#pragma unroll
                for (int k = 0; k < 32; ++k) gc[k] = G[k];
            }
#pragma unroll
            for (int s = 0; s < SUB; ++s) apply_op_g<T, R>(vr[s], vi[s], i1, g1);
        }
    }
    if (nops & 1) {
#pragma unroll
        for (int k = 0; k < 32; ++k) gc[k] = g1[k];
    }
}

// The same with the gates in vector registers, read from the workgroup's LDS
// copy of the gate table (lg, 32 floats per gate): FP32 FMAs whose operands
// all sit in vector registers can issue two per cycle per SIMD on gfx950 when
// two waves have one ready, where an FMA that reads a scalar register issues
// alone.  All lanes read the same address, so each 16-byte read is a
// broadcast.
template <typename T, int R, int SUB>
__device__ __forceinline__ void sweep_group_ops_lg(T (&vr)[SUB][1 << R], T (&vi)[SUB][1 << R], const fl_pass& pd,
                                                   int g, const float* lg) {
    const int nops = pass_nops(pd, g);
    // op metadata (bit, gate index) is read with scalar loads one op ahead;
    // LDS and scalar loads share one wait counter, so the next op's scalar
    // loads are issued only after this op's gate has arrived from LDS, and
    // they complete under the op's FMAs.
    int bit = pass_bit(pd, g, 0), idx = pass_gate(pd, g, 0);
    auto run = [&](int q) {
        __builtin_amdgcn_s_waitcnt(FL_WAIT_LGKM0);
        const float4* src = reinterpret_cast<const float4*>(lg + 32 * idx);
        T gv[32];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const float4 v = src[k];
            gv[4 * k] = v.x;
            gv[4 * k + 1] = v.y;
            gv[4 * k + 2] = v.z;
            gv[4 * k + 3] = v.w;
        }
        __builtin_amdgcn_s_waitcnt(FL_WAIT_LGKM0);
        const int i = bit;
        const int qn = q + 1 < nops ? q + 1 : q;
        bit = pass_bit(pd, g, qn);
        idx = pass_gate(pd, g, qn);
#pragma unroll
        for (int s = 0; s < SUB; ++s) apply_op_g<T, R>(vr[s], vi[s], i, gv);
    };
    for (int q = 0; q < nops; q += 2) {
        run(q);
        if (q + 1 < nops) run(q + 1);
    }
}

// Full-size tiles (K = KT), one tile per workgroup.  Every thread holds SUB
// register groups of 2^R amplitudes and applies each gate to all of them.
// With LG (complex64) each op reads its gate from the workgroup's LDS copy of
// the gate table into vector registers; otherwise (complex128) the next
// gate's matrix is fetched into scalar registers while the current one is
// applied.
//
// The first group is loaded straight from HBM into its register layout, and
// the last group stored straight back, when the group's lowest bit u0 is at
// least FL_DIRECT_MIN_U0: the lanes then still cover runs of >= 2^4
// contiguous amplitudes (>= 128 bytes), so every access coalesces.  This
// saves one LDS round trip and one barrier at each end of the pass.  Groups
// starting lower go through the LDS transpose, as every middle group does.
//
// LDS slots of 13-bit complex64 tiles with 5-bit register groups (the bond
// reduction's layout, and the sweep's with 256-thread workgroups).  Each run
// of 16 lanes of an 8-byte LDS access must hit 16 distinct slots modulo 16.
// In a register group with first bit u0 the 16 lanes vary the four lowest
// tile bits outside [u0, u0 + 5): bits 5..8 for u0 = 0, {0, 6, 7, 8} for
// u0 = 1, and so on.  fl_swz (bits 4..7 into bits 0..3) misses bit 8 and gives
// two-way conflicts for u0 < 4; XOR-ing bits 5..8 into bits 0..3 and bit 4
// into bit 0 keeps every one of these patterns and the pairwise tile
// loads (lanes varying bits 1..4) conflict-free.  Like fl_swz it is linear
// over XOR, its added term depends on none of bits 0..3, and it leaves every
// bit from 9 up alone.
// Sweeps with 4-bit register groups (complex64 with 512-thread workgroups,
// complex128) keep fl_swz, which serves every u0 of a 4-bit group.
template <typename T, int R>
__device__ __forceinline__ uint32_t sweep_swz(uint32_t j) {
    if constexpr (sizeof(T) == 4 && R == 5) return j ^ ((j >> 5) & 15u) ^ ((j >> 4) & 1u);
    else return fl_swz(j);
}

template <typename T, int R, int KT, int NT, int CL, bool LG>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(NT * 2 / 256))) void k_sweep_tiles(typename CT<T>::c* __restrict__ psi,
                                                    const T* __restrict__ gates, int W, fl_pass pd, int ngates) {
    typedef typename CT<T>::c cplx;
    static_assert(!LG || sizeof(T) == 4, "LDS gate table: complex64 only");
    __shared__ __attribute__((aligned(16))) float lg[LG ? FL_MAX_GATE_TABLE * 32 : 4];
    if constexpr (LG) {
        const float4* src = reinterpret_cast<const float4*>(gates);
        for (int t = threadIdx.x; t < ngates * 8; t += NT) reinterpret_cast<float4*>(lg)[t] = src[t];
    }
    constexpr int C = CL;
    static_assert(C >= FL_DIRECT_MIN_U0, "direct register transfers need 2^FL_DIRECT_MIN_U0 contiguous amplitudes");
    constexpr int K = KT;
    constexpr int SUB = (1 << (K - R)) / NT;
    static_assert(SUB >= 1, "tile too small for the workgroup");
    constexpr int APL = (sizeof(T) == 4) ? 2 : 1;           // amplitudes per 16-byte access
    constexpr int ITER = (1 << K) / (APL * NT);
    typedef typename std::conditional<sizeof(T) == 4, float4, double2>::type v16;
    __shared__ cplx lds[1 << K];
    const int h = pd.h;
    const int ng = pd.ngroups;
    cplx* const base = psi + fl_tile_base(blockIdx.x, C, W, h);
    // Element j = APL (tid + s NT) of a tile sits at toff + s * tstride: APL NT
    // is a multiple of 2^C, so s only moves the window part of the offset.
    static_assert((APL * NT) % (1 << C) == 0 && (APL * NT) % 256 == 0, "tile access stride");
    const uint64_t toff = fl_tile_offset(APL * threadIdx.x, C, h);
    const uint64_t tstride = (uint64_t)((APL * NT) >> C) << h;
    // LDS slot of element j + s APL NT is sweep_swz(j) + s APL NT (the
    // swizzle only mixes bits 0..8), and sweep_swz(j + 1) = sweep_swz(j) ^ 1
    // for even j.
    const uint32_t l0 = sweep_swz<T, R>(APL * threadIdx.x);
    const bool din = ng > 0 && pass_u0(pd, 0) >= FL_DIRECT_MIN_U0;
    const bool dout = ng > 0 && pass_u0(pd, ng - 1) >= FL_DIRECT_MIN_U0;

    T vr[SUB][1 << R], vi[SUB][1 << R];
    uint32_t b0[SUB];
    // HBM offsets of a register group: element b0 | (m << u0) of the tile sits
    // at off(b0) + sum over the set bits k of m of d[k].
    auto group_offsets = [&](int u0, uint64_t (&o)[SUB], uint64_t (&d)[R]) {
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const int q = u0 + k;
            d[k] = q < C ? (1ull << q) : (1ull << (h + q - C));
        }
#pragma unroll
        for (int s = 0; s < SUB; ++s) {
            b0[s] = fl_spread(threadIdx.x + s * NT, u0, R);
            o[s] = fl_tile_offset(b0[s], C, h);
        }
    };
    auto moff = [&](const uint64_t (&d)[R], int m) {
        uint64_t r = 0;
#pragma unroll
        for (int k = 0; k < R; ++k)
            if ((m >> k) & 1) r += d[k];
        return r;
    };
    // LDS byte offsets of the current register group.  The swizzle is linear
    // over XOR and b0 and m << u0 have disjoint bits, so
    // slot(b0 | m << u0) = slot(b0) ^ slot(m << u0), and slot(m << u0) is the
    // XOR of the (uniform) slots of m's set bits: one VALU XOR per element.
    // Kept for the group's write-back.
    uint32_t la[SUB][1 << R];
    auto lds_addrs = [&](int u0) {
        uint32_t bk[R];
#pragma unroll
        for (int k = 0; k < R; ++k) bk[k] = sweep_swz<T, R>(1u << (u0 + k)) * (uint32_t)sizeof(cplx);
#pragma unroll
        for (int s = 0; s < SUB; ++s) {
            b0[s] = fl_spread(threadIdx.x + s * NT, u0, R);
            la[s][0] = sweep_swz<T, R>(b0[s]) * (uint32_t)sizeof(cplx);
#pragma unroll
            for (int m = 1; m < (1 << R); ++m) la[s][m] = la[s][m & (m - 1)] ^ bk[__builtin_ctz(m)];
        }
    };
    char* const lbytes = reinterpret_cast<char*>(lds);
    auto lds_to_regs = [&]() {
#pragma unroll
        for (int s = 0; s < SUB; ++s)
#pragma unroll
            for (int m = 0; m < (1 << R); ++m) {
                const cplx a = *reinterpret_cast<const cplx*>(lbytes + la[s][m]);
                vr[s][m] = a.x;
                vi[s][m] = a.y;
            }
    };
    auto regs_to_lds = [&]() {
#pragma unroll
        for (int s = 0; s < SUB; ++s)
#pragma unroll
            for (int m = 0; m < (1 << R); ++m) {
                cplx a;
                a.x = vr[s][m];
                a.y = vi[s][m];
                *reinterpret_cast<cplx*>(lbytes + la[s][m]) = a;
            }
    };

    if (din) {
        uint64_t o[SUB], d[R];
        group_offsets(pass_u0(pd, 0), o, d);
#pragma unroll
        for (int s = 0; s < SUB; ++s)
#pragma unroll
            for (int m = 0; m < (1 << R); ++m) {
                const cplx a = base[o[s] + moff(d, m)];
                vr[s][m] = a.x;
                vi[s][m] = a.y;
            }
    } else {
        v16 nxt[ITER];
#pragma unroll
        for (int s = 0; s < ITER; ++s) nxt[s] = *reinterpret_cast<const v16*>(base + toff + s * tstride);
#pragma unroll
        for (int s = 0; s < ITER; ++s) {
            const uint32_t l = l0 + s * (APL * NT);
            if constexpr (sizeof(T) == 4) {
                lds[l] = make_float2(nxt[s].x, nxt[s].y);
                lds[l ^ 1] = make_float2(nxt[s].z, nxt[s].w);
            } else {
                lds[l] = nxt[s];
            }
        }
        __syncthreads();
        if (ng > 0) {
            lds_addrs(pass_u0(pd, 0));
            lds_to_regs();
        }
    }

    // the first gate of the pass (later groups find theirs fetched by the
    // previous group's op loop)
    T gx[32];
    if (!LG && ng > 0) {
        const T* G = gates + 32 * pass_gate(pd, 0, 0);
#pragma unroll
        for (int k = 0; k < 32; ++k) gx[k] = G[k];
    }
    if (LG && din) __syncthreads();   // the gate table (other paths pass a barrier after the tile load)
    for (int g = 0; g < ng; ++g) {
        const int u0 = pass_u0(pd, g);
        if (g > 0 || din) lds_addrs(u0);
        if (g > 0) lds_to_regs();
        if constexpr (LG)
            sweep_group_ops_lg<T, R, SUB>(vr, vi, pd, g, lg);
        else
            sweep_group_ops<T, R, SUB>(vr, vi, pd, g, gates, gx);
        if (g == ng - 1 && dout) break;
        regs_to_lds();
        __syncthreads();
    }

    if (dout) {
        uint64_t o[SUB], d[R];
        group_offsets(pass_u0(pd, ng - 1), o, d);
#pragma unroll
        for (int s = 0; s < SUB; ++s)
#pragma unroll
            for (int m = 0; m < (1 << R); ++m) {
                cplx a;
                a.x = vr[s][m];
                a.y = vi[s][m];
                base[o[s] + moff(d, m)] = a;
            }
    } else {
#pragma unroll
        for (int s = 0; s < ITER; ++s) {
            const uint32_t l = l0 + s * (APL * NT);
            if constexpr (sizeof(T) == 4) {
                const float2 a = lds[l], b = lds[l ^ 1];
                *reinterpret_cast<float4*>(base + toff + s * tstride) = make_float4(a.x, a.y, b.x, b.y);
            } else {
                *reinterpret_cast<v16*>(base + toff + s * tstride) = lds[l];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// wave-level reductions
// ---------------------------------------------------------------------------

// NV values per lane -> lane l returns the wave-wide sum of value index
// l >> (6 - log2 NV).  Each step keeps one half of the values and trades the
// other half with the partner lane, so the whole reduction costs
// NV/2 + NV/4 + ... shuffles instead of NV * 6.  Written as a template
// recursion so that every array index is a compile-time constant.
// FP32 form on gfx950: the first two steps are one v_permlane32_swap /
// v_permlane16_swap per value pair (the swap trades exactly the half that the
// partner keeps, so x' + y' is the step's result without any select), the
// distance-8 step moves the sent half by DPP row_ror:8 (= lane ^ 8 inside a
// row of 16), and the final in-quad steps use DPP quad_perm.
template <int CTRL>
__device__ __forceinline__ float fl_dpp_f(float x) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), CTRL, 0xf, 0xf, false));
}

template <int N, int D>
__device__ __forceinline__ void tr_steps_f32(float (&v)[N], int lane) {
    if constexpr (N > 1) {
        constexpr int H = N / 2;
#pragma unroll
        for (int k = 0; k < H; ++k) {
            if constexpr (D == 32 || D == 16) {
                const auto r = (D == 32) ? __builtin_amdgcn_permlane32_swap(__float_as_uint(v[k]),
                                                                            __float_as_uint(v[k + H]), false, false)
                                         : __builtin_amdgcn_permlane16_swap(__float_as_uint(v[k]),
                                                                            __float_as_uint(v[k + H]), false, false);
                v[k] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
            } else {
                const bool upper = (lane & D) != 0;
                const float keep = upper ? v[k + H] : v[k];
                const float send = upper ? v[k] : v[k + H];
                // D = 8: row_ror:8 pairs lane i with i ^ 8.  D = 4:
                // row_half_mirror pairs lane i with 7 - i in its run of 8; any
                // pairing of the lanes with bit 2 clear to those with it set
                // serves, the later steps sum over the whole run.
                float got;
                if constexpr (D == 8)
                    got = fl_dpp_f<0x128>(send);
                else if constexpr (D == 4)
                    got = fl_dpp_f<0x141>(send);
                else
                    got = __shfl_xor(send, D);
                v[k] = keep + got;
            }
        }
        tr_steps_f32<H, D / 2>(*reinterpret_cast<float(*)[H]>(&v[0]), lane);
    } else {
        if constexpr (D >= 32) v[0] += __shfl_xor(v[0], 32);
        if constexpr (D >= 16) v[0] += __shfl_xor(v[0], 16);
        if constexpr (D >= 8) v[0] += fl_dpp_f<0x128>(v[0]);
        if constexpr (D >= 4) v[0] += fl_dpp_f<0x141>(v[0]);  // row_half_mirror: lane 7 - i of the run of 8
        if constexpr (D >= 2) v[0] += fl_dpp_f<0x4E>(v[0]);   // quad_perm(2,3,0,1): lane ^ 2
        if constexpr (D >= 1) v[0] += fl_dpp_f<0xB1>(v[0]);   // quad_perm(1,0,3,2): lane ^ 1
    }
}

// FP64 form: the same lane pattern as tr_steps_f32, moving each double as its
// two 32-bit halves (two permlane swaps or two DPP moves per value); the adds
// are FP64.
template <int CTRL>
__device__ __forceinline__ double fl_dpp_d(double x) {
    const uint64_t u = (uint64_t)__double_as_longlong(x);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)u, CTRL, 0xf, 0xf, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)(u >> 32), CTRL, 0xf, 0xf, false);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

template <int N, int D>
__device__ __forceinline__ void tr_steps_f64(double (&v)[N], int lane) {
    if constexpr (N > 1) {
        constexpr int H = N / 2;
#pragma unroll
        for (int k = 0; k < H; ++k) {
            if constexpr (D == 32 || D == 16) {
                const uint64_t a = (uint64_t)__double_as_longlong(v[k]), b = (uint64_t)__double_as_longlong(v[k + H]);
                const auto rl = (D == 32) ? __builtin_amdgcn_permlane32_swap((uint32_t)a, (uint32_t)b, false, false)
                                          : __builtin_amdgcn_permlane16_swap((uint32_t)a, (uint32_t)b, false, false);
                const auto rh = (D == 32)
                                    ? __builtin_amdgcn_permlane32_swap((uint32_t)(a >> 32), (uint32_t)(b >> 32), false, false)
                                    : __builtin_amdgcn_permlane16_swap((uint32_t)(a >> 32), (uint32_t)(b >> 32), false, false);
                const double x = __longlong_as_double((long long)(((uint64_t)rh[0] << 32) | rl[0]));
                const double y = __longlong_as_double((long long)(((uint64_t)rh[1] << 32) | rl[1]));
                v[k] = x + y;
            } else {
                const bool upper = (lane & D) != 0;
                const double keep = upper ? v[k + H] : v[k];
                const double send = upper ? v[k] : v[k + H];
                double got;
                if constexpr (D == 8)
                    got = fl_dpp_d<0x128>(send);
                else if constexpr (D == 4)
                    got = fl_dpp_d<0x141>(send);
                else
                    got = __shfl_xor(send, D);
                v[k] = keep + got;
            }
        }
        tr_steps_f64<H, D / 2>(*reinterpret_cast<double(*)[H]>(&v[0]), lane);
    } else {
        if constexpr (D >= 32) v[0] += __shfl_xor(v[0], 32);
        if constexpr (D >= 16) v[0] += __shfl_xor(v[0], 16);
        if constexpr (D >= 8) v[0] += fl_dpp_d<0x128>(v[0]);
        if constexpr (D >= 4) v[0] += fl_dpp_d<0x141>(v[0]);
        if constexpr (D >= 2) v[0] += fl_dpp_d<0x4E>(v[0]);
        if constexpr (D >= 1) v[0] += fl_dpp_d<0xB1>(v[0]);
    }
}

template <typename T, int NV>
__device__ __forceinline__ T wave_transpose_reduce(T (&v)[NV]) {
    static_assert(NV >= 1 && NV <= 64 && (NV & (NV - 1)) == 0, "NV must be a power of two <= 64");
    if constexpr (sizeof(T) == 4)
        tr_steps_f32<NV, 32>(v, threadIdx.x & 63);
    else
        tr_steps_f64<NV, 32>(v, threadIdx.x & 63);
    return v[0];
}

// ---------------------------------------------------------------------------
// reduced density matrices of the bonds of a cover pass (+ norm)
// ---------------------------------------------------------------------------
// Per bond: rho[i][j] = sum_r psi_{r,i} conj(psi_{r,j}); stored as 16 reals:
// [0..3] = rho_ii, then (re, im) of rho_01, rho_02, rho_03, rho_12, rho_13, rho_23.
// partials layout: [gridDim.x][nslot][16] doubles, slot = bond, slot L-1 = norm.

#define FL_RDM_MAXG 16
#define FL_RDM_TILE_MAXG 13   // bond slots of a full-tile cover pass (K-1 <= 12) + the norm

// Adds one quad (amplitudes a_0..a_3 of a bond's local index) to the 16
// density-matrix sums: [0..3] |a_l|^2, then for each pair l < m the real and
// imaginary parts of conj(a_l) a_m (as ar_l ar_m + ai_l ai_m and
// ai_l ar_m - ar_l ai_m), pairs in the order 01, 02, 03, 12, 13, 23.
template <typename T>
__device__ __forceinline__ void rdm_quad(const T (&ar)[4], const T (&ai)[4], T (&r)[16]) {
#pragma unroll
    for (int l = 0; l < 4; ++l) r[l] = fma(ar[l], ar[l], fma(ai[l], ai[l], r[l]));
    int k = 4;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = i + 1; j < 4; ++j) {
            r[k] = fma(ar[i], ar[j], fma(ai[i], ai[j], r[k]));
            r[k + 1] = fma(ai[i], ar[j], fma(-ar[i], ai[j], r[k + 1]));
            k += 2;
        }
}

template <typename T, int KT, int KMAX>
__global__ __launch_bounds__(FL_NT) void k_rdm(const typename CT<T>::c* __restrict__ psi, int C, int W,
                                               uint32_t ntiles, fl_pass pd, double* __restrict__ partials,
                                               int nslot) {
    typedef typename CT<T>::c cplx;
    __shared__ cplx lds[1 << KMAX];
    __shared__ double wacc[FL_NT / 64][FL_RDM_MAXG + 1][16];
    const int K = KT > 0 ? KT : C + W;
    const int h = pd.h;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double acc[FL_RDM_MAXG];
#pragma unroll
    for (int g = 0; g < FL_RDM_MAXG; ++g) acc[g] = 0.0;
    double nrm = 0.0;
    const uint32_t ngrp = 1u << (K - 2);
    for (uint32_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const uint64_t base = fl_tile_base(tile, C, W, h);
        __syncthreads();
        tile_load<T, KT>(psi, base, K, C, h, lds);
        __syncthreads();
        if (pd.flags & 1) {
            for (uint32_t j = threadIdx.x; j < (1u << K); j += FL_NT) {
                const cplx a = lds[fl_swz(j)];
                nrm += (double)a.x * (double)a.x + (double)a.y * (double)a.y;
            }
        }
#pragma unroll
        for (int g = 0; g < FL_RDM_MAXG; ++g) {
            if (g < pd.ngroups) {
                const int u = pd.u0[g];
                double r[16];
#pragma unroll
                for (int k = 0; k < 16; ++k) r[k] = 0.0;
                for (uint32_t o = threadIdx.x; o < ngrp; o += FL_NT) {
                    const uint32_t b0 = fl_spread(o, u, 2);
                    double ar[4], ai[4];
#pragma unroll
                    for (int l = 0; l < 4; ++l) {
                        const cplx a = lds[fl_swz(b0 | ((uint32_t)l << u))];
                        ar[l] = a.x;
                        ai[l] = a.y;
                    }
#pragma unroll
                    for (int l = 0; l < 4; ++l) r[l] = fma(ar[l], ar[l], fma(ai[l], ai[l], r[l]));
                    int k = 4;
#pragma unroll
                    for (int i = 0; i < 4; ++i)
#pragma unroll
                        for (int j = i + 1; j < 4; ++j) {
                            r[k] = fma(ar[i], ar[j], fma(ai[i], ai[j], r[k]));
                            r[k + 1] = fma(ai[i], ar[j], fma(-ar[i], ai[j], r[k + 1]));
                            k += 2;
                        }
                }
                acc[g] += wave_transpose_reduce<double, 16>(r);
            }
        }
    }
    // per-wave accumulators -> LDS -> one row of partials per workgroup
    double nv[1] = {nrm};
    const double ntot = wave_transpose_reduce<double, 1>(nv);
    if ((lane & 3) == 0) {
#pragma unroll
        for (int g = 0; g < FL_RDM_MAXG; ++g) wacc[wave][g][lane >> 2] = acc[g];
    }
    if (lane == 0) wacc[wave][FL_RDM_MAXG][0] = ntot;
    __syncthreads();
    for (int t = threadIdx.x; t < (pd.ngroups + 1) * 16; t += FL_NT) {
        const int g = t >> 4, v = t & 15;
        const int gg = (g < pd.ngroups) ? g : FL_RDM_MAXG;
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < FL_NT / 64; ++w) s += wacc[w][gg][v];
        if (g < pd.ngroups) {
            partials[((size_t)blockIdx.x * nslot + pd.ops[g][0]) * 16 + v] = s;
        } else if ((pd.flags & 1) && v == 0) {
            partials[((size_t)blockIdx.x * nslot + (nslot - 1)) * 16] = s;
        }
    }
}

// Full-size tiles: persistent workgroups with the next tile prefetched into
// registers (as in k_sweep_tiles).  All sums are FP64: complex64 amplitudes
// are widened to FP64, so every product of two of them is exact and only the
// FP64 additions round; complex128 states use FP64 throughout.
template <typename T, int KT, int NT>
__global__ __launch_bounds__(NT) void k_rdm_tiles(const typename CT<T>::c* __restrict__ psi, int W, uint32_t ntiles,
                                                  fl_pass pd, double* __restrict__ partials, int nslot) {
    typedef typename CT<T>::c cplx;
    constexpr int C = FL_LOWBITS;
    constexpr int K = KT;
    constexpr int APL = (sizeof(T) == 4) ? 2 : 1;
    constexpr int ITER = (1 << K) / (APL * NT);
    constexpr int NW = NT / 64;
    constexpr int NG = FL_RDM_TILE_MAXG;
    typedef typename std::conditional<sizeof(T) == 4, float4, double2>::type v16;
    __shared__ cplx lds[1 << K];
    __shared__ double wacc[NW][NG][16];
    const int h = pd.h;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int t = threadIdx.x; t < NW * NG * 16; t += NT) (&wacc[0][0][0])[t] = 0.0;
    double nrm = 0.0;
    static_assert((APL * NT) % (1 << C) == 0 && (APL * NT) % 256 == 0, "tile access stride");
    const uint64_t toff = fl_tile_offset(APL * threadIdx.x, C, h);
    const uint64_t tstride = (uint64_t)((APL * NT) >> C) << h;
    for (uint32_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const cplx* src = psi + fl_tile_base(tile, C, W, h) + toff;
        v16 v[ITER];
#pragma unroll
        for (int s = 0; s < ITER; ++s) v[s] = *reinterpret_cast<const v16*>(src + s * tstride);
        __syncthreads();
#pragma unroll
        for (int s = 0; s < ITER; ++s) {
            const uint32_t j = APL * (threadIdx.x + s * NT);
            if constexpr (sizeof(T) == 4) {
                lds[fl_swz(j)] = make_float2(v[s].x, v[s].y);
                lds[fl_swz(j + 1)] = make_float2(v[s].z, v[s].w);
                nrm = fma((double)v[s].x, (double)v[s].x, fma((double)v[s].y, (double)v[s].y, nrm));
                nrm = fma((double)v[s].z, (double)v[s].z, fma((double)v[s].w, (double)v[s].w, nrm));
            } else {
                lds[fl_swz(j)] = v[s];
                nrm = fma(v[s].x, v[s].x, fma(v[s].y, v[s].y, nrm));
            }
        }
        __syncthreads();
        for (int g = 0; g < pd.ngroups; ++g) {
            const int u = pass_u0(pd, g);
            double r[16];
#pragma unroll
            for (int k = 0; k < 16; ++k) r[k] = 0.0;
            // slot(spread(tid + NT s) | l << u) = slot(spread(tid)) ^ slot(spread(NT s)) ^ slot(l << u)
            // (the swizzle is linear over XOR; the three parts have disjoint
            // bits), the last two uniform: one VALU XOR per read
            const uint32_t vb = fl_swz(fl_spread(threadIdx.x, u, 2)) * (uint32_t)sizeof(cplx);
            constexpr int NS = (1 << (K - 2)) / NT;
            // all reads of the group first, so that their latencies overlap
            cplx q[NS][4];
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                const uint32_t us = fl_swz(fl_spread((uint32_t)(s * NT), u, 2)) * (uint32_t)sizeof(cplx);
#pragma unroll
                for (int l = 0; l < 4; ++l) {
                    const uint32_t ul = us ^ (fl_swz((uint32_t)l << u) * (uint32_t)sizeof(cplx));
                    q[s][l] = *reinterpret_cast<const cplx*>(reinterpret_cast<const char*>(lds) + (vb ^ ul));
                }
            }
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                double ar[4], ai[4];
#pragma unroll
                for (int l = 0; l < 4; ++l) {
                    ar[l] = (double)q[s][l].x;
                    ai[l] = (double)q[s][l].y;
                }
                rdm_quad<double>(ar, ai, r);
            }
            // lane l holds the sum of value l >> 2; one lane of each four adds
            // it, the others add zero (an LDS atomic with every lane active)
            const double red = wave_transpose_reduce<double, 16>(r);
            __hip_atomic_fetch_add(&wacc[wave][g][lane >> 2], (lane & 3) == 0 ? red : 0.0, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
        }
    }
    double nv[1] = {nrm};
    const double ntot = wave_transpose_reduce<double, 1>(nv);
    __syncthreads();
    if (lane == 0) wacc[wave][NG - 1][0] = ntot;   // the norm uses the last slot row
    __syncthreads();
    for (int t = threadIdx.x; t < (pd.ngroups + 1) * 16; t += NT) {
        const int g = t >> 4, v = t & 15;
        const int gg = (g < pd.ngroups) ? g : NG - 1;
        if (g == pd.ngroups && v > 0) continue;
        double sum = 0.0;
#pragma unroll
        for (int w = 0; w < NW; ++w) sum += wacc[w][gg][v];
        if (g < pd.ngroups) {
            partials[((size_t)blockIdx.x * nslot + pd.ops[g][0]) * 16 + v] = sum;
        } else if (pd.flags & 1) {
            partials[((size_t)blockIdx.x * nslot + (nslot - 1)) * 16] = sum;
        }
    }
}

template <int A, int B, typename F>
__device__ __forceinline__ void static_for(F&& f) {
    if constexpr (A < B) {
        f(std::integral_constant<int, A>{});
        static_for<A + 1, B>(f);
    }
}

// Density-matrix sums of the bond on register bits (I, I+1) of a register group.
template <int R, int I>
__device__ __forceinline__ void group_bond_sums(const double (&vr)[1 << R], const double (&vi)[1 << R], double (&r)[16]) {
    // (immediate-operand markers keep the bit variants apart, as in apply_pair_g)
    __asm__ volatile("; bond sums on register bits %0" ::"i"(I));
#pragma unroll
    for (int c = 0; c < (1 << R) / 4; ++c) {
        const int b = (c & ((1 << I) - 1)) | ((c >> I) << (I + 2));
        double ar[4], ai[4];
#pragma unroll
        for (int l = 0; l < 4; ++l) {
            ar[l] = vr[b | (l << I)];
            ai[l] = vi[b | (l << I)];
        }
        rdm_quad<double>(ar, ai, r);
    }
    __asm__ volatile("; end bond sums on register bits %0" ::"i"(I));
}

// Bond reductions of complex64 states over full 13-bit tiles with 5-bit
// register groups (the layout of the complex64 sweep): a cover pass's bonds
// come packed into groups of R consecutive tile bits, every thread reads a
// group's 2^R amplitudes from LDS once and forms the sums of all the group's
// bonds from registers (8 quads per bond and thread), so each LDS word is read
// once per group rather than once per bond.  The group's amplitudes are
// widened to FP64 when they leave LDS, so each product of two FP32 values is
// exact; each lane sums its quads in FP64, the wave tree is FP64 and its
// result goes into FP64 per-wave LDS accumulators.  The norm is an FP64 sum
// as well.  Persistent workgroups; partials as in k_rdm_tiles.
template <int R, int KT, int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(NT * 2 / 256))) void k_rdm_groups(
    const float2* __restrict__ psi, int W, uint32_t ntiles, fl_pass pd, double* __restrict__ partials, int nslot) {
    constexpr int C = FL_LOWBITS;
    constexpr int K = KT;
    static_assert((1 << (K - R)) == NT, "one register group per thread");
    constexpr int ITER = (1 << K) / (2 * NT);
    constexpr int NW = NT / 64;
    constexpr int NS = FL_RDM_TILE_MAXG;   // bond rows (K - 1 at most) + the norm
    static_assert(K - 1 < NS, "bond rows");
    __shared__ __attribute__((aligned(16))) float2 lds[1 << K];
    __shared__ double wacc[NW][NS][16];
    const char* const lb = reinterpret_cast<const char*>(lds);
    const int h = pd.h;
    const int ng = pd.ngroups;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int t = threadIdx.x; t < NW * NS * 16; t += NT) (&wacc[0][0][0])[t] = 0.0;
    double nrm = 0.0;
    static_assert((2 * NT) % (1 << C) == 0, "tile access stride");
    // element 2 (tid + s NT) of a tile sits at toff + s tstride, LDS slot
    // sweep_swz(j) + s 2 NT, and sweep_swz(j + 1) = sweep_swz(j) ^ 1
    const uint64_t toff = fl_tile_offset(2 * threadIdx.x, C, h);
    const uint64_t tstride = (uint64_t)((2 * NT) >> C) << h;
    const uint32_t l0 = sweep_swz<float, R>(2 * threadIdx.x);
    for (uint32_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const float2* src = psi + fl_tile_base(tile, C, W, h) + toff;
        float4 v[ITER];
#pragma unroll
        for (int s = 0; s < ITER; ++s) {
            // streaming: each amplitude is read once per pass
            const fl_f32x4 t = __builtin_nontemporal_load(reinterpret_cast<const fl_f32x4*>(src + s * tstride));
            v[s] = make_float4(t[0], t[1], t[2], t[3]);
        }
        __syncthreads();   // the previous tile's LDS reads (and the accumulator reset) are done
#pragma unroll
        for (int s = 0; s < ITER; ++s) {
            const uint32_t l = l0 + s * (2 * NT);
            lds[l] = make_float2(v[s].x, v[s].y);
            lds[l ^ 1] = make_float2(v[s].z, v[s].w);
        }
        if (pd.flags & 1) {
#pragma unroll
            for (int s = 0; s < ITER; ++s) {
                nrm = fma((double)v[s].x, (double)v[s].x, fma((double)v[s].y, (double)v[s].y, nrm));
                nrm = fma((double)v[s].z, (double)v[s].z, fma((double)v[s].w, (double)v[s].w, nrm));
            }
        }
        __syncthreads();
        int row = 0;
        for (int g = 0; g < ng; ++g) {
            const int u0 = pass_u0(pd, g);
            const int nops = pass_nops(pd, g);
            // slot(b0 | m << u0) = slot(b0) ^ XOR of the slots of m's set bits
            uint32_t bk[R];
#pragma unroll
            for (int k = 0; k < R; ++k) bk[k] = sweep_swz<float, R>(1u << (u0 + k)) * 8u;
            uint32_t la[1 << R];
            la[0] = sweep_swz<float, R>(fl_spread(threadIdx.x, u0, R)) * 8u;
#pragma unroll
            for (int m = 1; m < (1 << R); ++m) la[m] = la[m & (m - 1)] ^ bk[__builtin_ctz(m)];
            double vr[1 << R], vi[1 << R];
#pragma unroll
            for (int m = 0; m < (1 << R); ++m) {
                const float2 a = *reinterpret_cast<const float2*>(lb + la[m]);
                vr[m] = (double)a.x;
                vi[m] = (double)a.y;
            }
            // the group's bonds sit on pair bits i (ops in increasing i): one
            // compile-time code block per pair position, run when present
            uint32_t present = 0;
            for (int k = 0; k < nops; ++k) present |= 1u << pass_bit(pd, g, k);
            static_for<0, R - 1>([&](auto I) {
                constexpr int i = decltype(I)::value;
                if ((present >> i) & 1u) {
                    double r[16];
#pragma unroll
                    for (int q = 0; q < 16; ++q) r[q] = 0.0;
                    group_bond_sums<R, i>(vr, vi, r);
                    // lane l holds the sum of value l >> 2; one lane of each four
                    // adds it, the others add zero (an LDS atomic with every lane active)
                    const double red = wave_transpose_reduce<double, 16>(r);
                    const int rw = row + __builtin_popcount(present & ((1u << i) - 1u));
                    __hip_atomic_fetch_add(&wacc[wave][rw][lane >> 2], (lane & 3) == 0 ? red : 0.0,
                                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                }
            });
            row += nops;
        }
    }
    double nv[1] = {nrm};
    const double ntot = wave_transpose_reduce<double, 1>(nv);
    __syncthreads();
    if (lane == 0) wacc[wave][NS - 1][0] = ntot;
    __syncthreads();
    // rows of the pass in group order -> partials[block][bond][16]
    int nrows = 0;
    for (int g = 0; g < ng; ++g) nrows += pass_nops(pd, g);
    for (int t = threadIdx.x; t < (nrows + 1) * 16; t += NT) {
        const int row = t >> 4, v = t & 15;
        if (row == nrows && v > 0) continue;
        const int rr = row < nrows ? row : NS - 1;
        double sum = 0.0;
#pragma unroll
        for (int w = 0; w < NW; ++w) sum += wacc[w][rr][v];
        if (row < nrows) {
            // the bond of row `row`: walk the groups
            int gg = 0, k = row;
            while (k >= pass_nops(pd, gg)) k -= pass_nops(pd, gg++);
            partials[((size_t)blockIdx.x * nslot + pd.ops[gg][k]) * 16 + v] = sum;
        } else if (pd.flags & 1) {
            partials[((size_t)blockIdx.x * nslot + (nslot - 1)) * 16] = sum;
        }
    }
}

// ---------------------------------------------------------------------------
// product state, overlap, finalize
// ---------------------------------------------------------------------------

template <typename T>
__global__ __launch_bounds__(256) void k_init(typename CT<T>::c* __restrict__ psi, const double2* __restrict__ tlo,
                                              const double2* __restrict__ tmid, const double2* __restrict__ thi,
                                              int a, int b, uint64_t n) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t x = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += stride) {
        const double2 p = thi[x >> (a + b)], q = tmid[(x >> a) & ((1ull << b) - 1ull)], r = tlo[x & ((1ull << a) - 1ull)];
        const double pr = p.x * q.x - p.y * q.y, pi = p.x * q.y + p.y * q.x;
        typename CT<T>::c o;
        o.x = (T)(pr * r.x - pi * r.y);
        o.y = (T)(pr * r.y + pi * r.x);
        psi[x] = o;
    }
}

// complex64 form: a thread writes amplitudes x, x + 1 (x even, one 16-byte
// store); they share the two high factors because the low table covers at
// least one bit.  Same FP64 arithmetic per amplitude as k_init.
__global__ __launch_bounds__(256) void k_init_pairs_c64(float4* __restrict__ psi2, const double2* __restrict__ tlo,
                                                       const double2* __restrict__ tmid,
                                                       const double2* __restrict__ thi, int a, int b, uint64_t n2) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n2; k += stride) {
        const uint64_t x = 2 * k;
        const double2 p = thi[x >> (a + b)], q = tmid[(x >> a) & ((1ull << b) - 1ull)];
        const double2 r0 = tlo[x & ((1ull << a) - 1ull)], r1 = tlo[(x + 1) & ((1ull << a) - 1ull)];
        const double pr = p.x * q.x - p.y * q.y, pi = p.x * q.y + p.y * q.x;
        float4 o;
        o.x = (float)(pr * r0.x - pi * r0.y);
        o.y = (float)(pr * r0.y + pi * r0.x);
        o.z = (float)(pr * r1.x - pi * r1.y);
        o.w = (float)(pr * r1.y + pi * r1.x);
        psi2[k] = o;
    }
}

template <typename TA, typename TB>
__global__ __launch_bounds__(256) void k_overlap(const typename CT<TA>::c* __restrict__ a,
                                                 const typename CT<TB>::c* __restrict__ b, uint64_t n,
                                                 double* __restrict__ partials) {
    __shared__ double wacc[4][4];
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t x = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += stride) {
        const double ar = a[x].x, ai = a[x].y, br = b[x].x, bi = b[x].y;
        v[0] = fma(ar, br, fma(ai, bi, v[0]));     // Re conj(a) b
        v[1] = fma(ar, bi, fma(-ai, br, v[1]));    // Im conj(a) b
        v[2] = fma(ar, ar, fma(ai, ai, v[2]));
        v[3] = fma(br, br, fma(bi, bi, v[3]));
    }
    const double r = wave_transpose_reduce<double, 4>(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if ((lane & 15) == 0) wacc[wave][lane >> 4] = r;
    __syncthreads();
    if (threadIdx.x < 4) {
        double s = 0.0;
        for (int w = 0; w < 4; ++w) s += wacc[w][threadIdx.x];
        partials[(size_t)blockIdx.x * 4 + threadIdx.x] = s;
    }
}

// One workgroup per output value: thread t sums partial rows t, t + 256, ...
// in order, then a fixed LDS tree adds the 256 thread sums, so the result
// does not depend on timing.
__global__ __launch_bounds__(256) void k_finalize(const double* __restrict__ partials, int nblocks, int nvals,
                                                  double* __restrict__ out) {
    __shared__ double red[256];
    const int v = blockIdx.x;
    double s = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += 256) s += partials[(size_t)b * nvals + v];
    red[threadIdx.x] = s;
    __syncthreads();
#pragma unroll
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[v] = red[0];
}

// <H0> = sum_b Re tr(h_b rho_b) from the finalized bond sums (Sec. IV,
// Eq. (10)), in FP64 on the device: thread b expands rho_b from its 16 reals
// and contracts it with h_b (FP64, row-major complex); thread 0 adds the bond
// terms in bond order.  out[0] = <H0>, out[1] = <psi|psi>; rdm (optional)
// receives every rho_b as 4x4 complex.  One workgroup of 64 threads, L <= 65.
__global__ __launch_bounds__(64) void k_energy_contract(const double* __restrict__ red, const double* __restrict__ h64,
                                                        int L, double* __restrict__ out, double* __restrict__ rdm) {
    __shared__ double trs[64];
    const int b = threadIdx.x;
    if (b < L - 1) {
        const double* v = red + (size_t)b * 16;
        double rr[16], ri[16];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            rr[5 * i] = v[i];
            ri[5 * i] = 0.0;
        }
        int k = 4;
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = i + 1; j < 4; ++j) {
                rr[4 * i + j] = v[k];
                ri[4 * i + j] = v[k + 1];
                rr[4 * j + i] = v[k];
                ri[4 * j + i] = -v[k + 1];
                k += 2;
            }
        const double* hb = h64 + (size_t)b * 32;
        double tr = 0.0;
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) tr += hb[2 * (4 * i + j)] * rr[4 * j + i] - hb[2 * (4 * i + j) + 1] * ri[4 * j + i];
        trs[b] = tr;
        if (rdm) {
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                rdm[(size_t)b * 32 + 2 * q] = rr[q];
                rdm[(size_t)b * 32 + 2 * q + 1] = ri[q];
            }
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double E = 0.0;
        for (int q = 0; q < L - 1; ++q) E += trs[q];
        out[0] = E;
        out[1] = red[(size_t)(L - 1) * 16];
    }
}

// ---------------------------------------------------------------------------
// lambda = H0 psi, out of place (the Hamiltonian application of Sec. V)
// ---------------------------------------------------------------------------
// One cover pass per launch; the first pass writes lambda, later passes add.

template <typename T, int KT, int KMAX>
__global__ __launch_bounds__(FL_NT) void k_apply_h(const typename CT<T>::c* __restrict__ psi,
                                                   typename CT<T>::c* __restrict__ lam, const T* __restrict__ hmat,
                                                   int C, int W, fl_pass pd, int first) {
    typedef typename CT<T>::c cplx;
    __shared__ cplx lp[1 << KMAX];
    __shared__ cplx ll[1 << KMAX];
    const int K = KT > 0 ? KT : C + W;
    const int h = pd.h;
    const uint64_t base = fl_tile_base(blockIdx.x, C, W, h);
    tile_load<T, KT>(psi, base, K, C, h, lp);
    if (first) {
        for (uint32_t j = threadIdx.x; j < (1u << K); j += FL_NT) {
            cplx z;
            z.x = 0;
            z.y = 0;
            ll[j] = z;
        }
    } else {
        tile_load<T, KT>(lam, base, K, C, h, ll);
    }
    __syncthreads();
    const uint32_t ngrp = 1u << (K - 2);
    for (int g = 0; g < pd.ngroups; ++g) {
        const int u = pd.u0[g];
        const T* H = hmat + 32 * pd.ops[g][0];
        for (uint32_t o = threadIdx.x; o < ngrp; o += FL_NT) {
            const uint32_t b0 = fl_spread(o, u, 2);
            T ar[4], ai[4];
#pragma unroll
            for (int l = 0; l < 4; ++l) {
                const cplx a = lp[fl_swz(b0 | ((uint32_t)l << u))];
                ar[l] = a.x;
                ai[l] = a.y;
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const uint32_t idx = fl_swz(b0 | ((uint32_t)i << u));
                cplx acc = ll[idx];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const T hr = H[8 * i + 2 * j], hi = H[8 * i + 2 * j + 1];
                    acc.x = fma(hr, ar[j], fma(-hi, ai[j], acc.x));
                    acc.y = fma(hr, ai[j], fma(hi, ar[j], acc.y));
                }
                ll[idx] = acc;
            }
        }
        __syncthreads();
    }
    tile_store<T, KT>(lam, base, K, C, h, ll);
}

// ---------------------------------------------------------------------------
// reverse pass of the gradient: undo gates on psi and lambda together
// ---------------------------------------------------------------------------
// Every op with a slot first accumulates, for its bond b on register bits
// (i, i+1), the anti-Hermitian overlap
//   D_b[i][j] += sum_r conj(lambda_{r,i}) psi_{r,j} - conj(psi_{r,i}) lambda_{r,j}
// (the only part of M_b = sum_r conj(lambda_{r,i}) psi_{r,j} that an
// anti-Hermitian gate derivative A = (dG) G^dagger sees), then applies the
// gate (G_b^dagger) to both states.  16 reals per bond:
// [0..3] = Im(conj(lambda_i) psi_i) summed, then (re, im) of D_01, D_02,
// D_03, D_12, D_13, D_23.
// Mpart layout: [gridDim.x][nbonds][16] doubles, accumulated across launches.

template <typename T, int R, int I>
__device__ __forceinline__ void adj_overlap(const T (&pr)[1 << R], const T (&pi)[1 << R], const T (&lr)[1 << R],
                                            const T (&li)[1 << R], T (&d)[16]) {
#pragma unroll
    for (int c = 0; c < (1 << (R - 2)); ++c) {
        const int b = (c & ((1 << I) - 1)) | ((c >> I) << (I + 2));
        T ar[4], ai[4], br[4], bi[4];   // a = lambda, b = psi
#pragma unroll
        for (int l = 0; l < 4; ++l) {
            ar[l] = lr[b | (l << I)];
            ai[l] = li[b | (l << I)];
            br[l] = pr[b | (l << I)];
            bi[l] = pi[b | (l << I)];
        }
#pragma unroll
        for (int l = 0; l < 4; ++l) d[l] = fma(ar[l], bi[l], fma(-ai[l], br[l], d[l]));
        int k = 4;
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
            for (int y = x + 1; y < 4; ++y) {
                T re = d[k], im = d[k + 1];
                re = fma(ar[x], br[y], re);
                re = fma(ai[x], bi[y], re);
                re = fma(-br[x], ar[y], re);
                re = fma(-bi[x], ai[y], re);
                im = fma(ar[x], bi[y], im);
                im = fma(-ai[x], br[y], im);
                im = fma(-br[x], ai[y], im);
                im = fma(bi[x], ar[y], im);
                d[k] = re;
                d[k + 1] = im;
                k += 2;
            }
    }
}

// One reverse op on register bits (I, I+1): the overlap terms of the op's
// slot (before the gate), then the gate on psi and on lambda.  Every op of a
// reverse plan has both a slot and a gate (the host checks this), so the
// variants hold no further branches.
template <typename T, int R, int I>
__device__ __forceinline__ void adj_op(T (&pr)[1 << R], T (&pi)[1 << R], T (&lr)[1 << R], T (&li)[1 << R],
                                       const T (&g)[32], T (&d)[16]) {
    __asm__ volatile("; adjoint op on register bits %0" ::"i"(I));
    adj_overlap<T, R, I>(pr, pi, lr, li, d);
    apply_pair_g<T, R, I>(pr, pi, g);
    apply_pair_g<T, R, I>(lr, li, g);
}

template <typename T, int R, int KT, int KMAX, int NT = FL_NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 && NT == FL_NT ? 2 : 1))) void k_adjoint(typename CT<T>::c* __restrict__ psi,
                                                   typename CT<T>::c* __restrict__ lam, const T* __restrict__ gates,
                                                   int C, int W, uint32_t ntiles, fl_pass pd,
                                                   double* __restrict__ Mpart, int nbonds) {
    typedef typename CT<T>::c cplx;
    __shared__ cplx lp[1 << KMAX];
    __shared__ cplx ll[1 << KMAX];
    __shared__ double wacc[NT / 64][FL_MAX_SLOTS][16];
    const int K = KT > 0 ? KT : C + W;
    const int h = pd.h;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int t = threadIdx.x; t < (NT / 64) * FL_MAX_SLOTS * 16; t += NT) (&wacc[0][0][0])[t] = 0.0;
    const uint32_t nsub = 1u << (K - R);   // <= NT
    const bool active = threadIdx.x < nsub;
    for (uint32_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const uint64_t base = fl_tile_base(tile, C, W, h);
        __syncthreads();
        tile_load<T, KT, NT>(psi, base, K, C, h, lp);
        tile_load<T, KT, NT>(lam, base, K, C, h, ll);
        __syncthreads();
        for (int g = 0; g < pd.ngroups; ++g) {
            const int u0 = pass_u0(pd, g);
            const int nops = pass_nops(pd, g);
            const uint32_t b0 = fl_spread(active ? threadIdx.x : 0u, u0, R);
            // byte offset of element b0 | m << u0: slot(b0) ^ slot(m << u0), the
            // second part uniform (the swizzle is linear over XOR)
            const uint32_t vb = fl_swz(b0) * (uint32_t)sizeof(cplx);
            auto loff = [&](int m) { return vb ^ (fl_swz((uint32_t)m << u0) * (uint32_t)sizeof(cplx)); };
            char* const pb = reinterpret_cast<char*>(lp);
            char* const lb = reinterpret_cast<char*>(ll);
            T pr[1 << R], pi[1 << R], lr[1 << R], li[1 << R];
#pragma unroll
            for (int m = 0; m < (1 << R); ++m) {
                const uint32_t o = loff(m);
                cplx a = *reinterpret_cast<const cplx*>(pb + o), b = *reinterpret_cast<const cplx*>(lb + o);
                if (!active) { a.x = a.y = b.x = b.y = 0; }
                pr[m] = a.x;
                pi[m] = a.y;
                lr[m] = b.x;
                li[m] = b.y;
            }
            // Ops run two per iteration with the op metadata read as scalar
            // words and the gate fetched into scalar registers one op ahead
            // (the structure of the forward sweep's op loop).
            auto fetch = [&](int q, int& i, int& slot, T (&gg)[32]) {
                i = pass_bit(pd, g, q);
                slot = pass_slot(pd, g, q);
                const T* G = gates + 32 * pass_gate(pd, g, q);
#pragma unroll
                for (int k = 0; k < 32; ++k) gg[k] = G[k];
            };
            auto run = [&](int i, int slot, const T (&gg)[32]) {
                T d[16];
#pragma unroll
                for (int k = 0; k < 16; ++k) d[k] = 0;
                with_bit<R>(i, [&](auto I) { adj_op<T, R, decltype(I)::value>(pr, pi, lr, li, gg, d); });
                // lane l holds the sum of value l >> 2; one lane of each
                // four adds it and the other three add zero, as an LDS atomic
                // with every lane active (no divergent branch in the op loop)
                const T r = wave_transpose_reduce<T, 16>(d);
                __hip_atomic_fetch_add(&wacc[wave][slot][lane >> 2], (lane & 3) == 0 ? (double)r : 0.0,
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            };
            int i0, s0;
            T gc[32];
            fetch(0, i0, s0, gc);
            for (int q = 0; q < nops; q += 2) {
                __builtin_amdgcn_s_waitcnt(FL_WAIT_LGKM0);
                int i1, s1;
                T gn[32];
                fetch((q + 1 < nops) ? q + 1 : q, i1, s1, gn);
                run(i0, s0, gc);
                if (q + 1 < nops) {
                    __builtin_amdgcn_s_waitcnt(FL_WAIT_LGKM0);
                    fetch((q + 2 < nops) ? q + 2 : q + 1, i0, s0, gc);
                    run(i1, s1, gn);
                }
            }
            if (active) {
#pragma unroll
                for (int m = 0; m < (1 << R); ++m) {
                    const uint32_t o = loff(m);
                    cplx a, b;
                    a.x = pr[m];
                    a.y = pi[m];
                    b.x = lr[m];
                    b.y = li[m];
                    *reinterpret_cast<cplx*>(pb + o) = a;
                    *reinterpret_cast<cplx*>(lb + o) = b;
                }
            }
            __syncthreads();
        }
        tile_store<T, KT, NT>(psi, base, K, C, h, lp);
        tile_store<T, KT, NT>(lam, base, K, C, h, ll);
    }
    __syncthreads();
    for (int t = threadIdx.x; t < pd.nslots * 16; t += NT) {
        const int sl = t >> 4, v = t & 15;
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < NT / 64; ++w) s += wacc[w][sl][v];
        double* dst = Mpart + ((size_t)blockIdx.x * nbonds + pd.sbond[sl]) * 16 + v;
        *dst += s;
    }
}

// The reverse pass of the gradient for the 4-qubit-window form (complex64,
// full 13-bit tiles), on the matrix cores.  The forward pass of that form
// applies, per register group (a 4-bit window whose ops q = 0 .. n-1 apply
// G_q inside the window), the FP32 real form of U = G_{n-1} ... G_0.  This
// kernel replays the same passes backwards, groups in reverse order, with the
// transposes of those FP32 matrices, i.e. the exact adjoints U^dagger of what
// the forward applied, so psi retraces the forward's states up to arithmetic
// rounding (as the plain form's replay with the adjoints of its FP32 gates
// does) and a reset from a checkpoint does not jump.  Per group:
//  - the window overlap Q[x][y] = sum_r psi_{r,x} conj(lambda_{r,y}) of the
//    state after the forward group, as the real 32 x 32 product
//    D[2x + a][2y + b] = sum_c psi_{x,a}(c) lambda_{y,b}(c) over the wave's
//    64 columns c (a, b = re, im) on v_mfma_f32_32x32x2f32: lane l supplies
//    row i = l % 32 of psi and column j = l % 32 of lambda at column k = l / 32
//    of the step, the same LDS position in both tiles.  Then
//    Re Q = D[2x][2y] + D[2x+1][2y+1] and Im Q = D[2x+1][2y] - D[2x][2y+1],
//    formed between neighbouring lanes and summed over the workgroup's tiles
//    in LDS (FP32, one 2 KiB row per group of the pass).  Every forward op's
//    bond overlap follows from Q: with the reverse ops r = 0 .. n-1 applying
//    G_{n-1-r}^dagger, the state before reverse op r is P_r Q P_r^dagger
//    (P_r the product of the reverse ops before it), traced over the two
//    window bits off the bond; the host forms these terms in FP64;
//  - U^dagger on psi and on lambda as in k_dense4 (mats: 4 KiB of A fragments
//    per group of the reverse pass, B = a 32-column block of the state).
// Wave w owns columns 64 w .. 64 w + 63 of the group (column = the tile bits
// off the window, in order) for both parts, so a barrier is needed only where
// the next group assigns the tile's elements to the waves differently.  The
// tiles use the slots of fl_swz12, under which the Q reads (lanes along the
// window's amplitudes) and the column reads meet at most two distinct
// addresses per bank.  At the end Qpart[blockIdx][g][0..255] = Re Q[x][y] at
// 16 x + y, [256..511] = Im Q (FP64 copies of the FP32 sums).
__global__ __launch_bounds__(FL_WIN4_NT) __attribute__((amdgpu_waves_per_eu(2))) void k_adjoint_win4(
    float2* __restrict__ psi, float2* __restrict__ lam, const float4* __restrict__ mats, int W, uint32_t ntiles,
    fl_pass pd, double* __restrict__ Qpart) {
    constexpr int K = FL_KMAX_C64;
    constexpr int C = FL_DENSE4_LOWBITS;
    constexpr int NT = FL_WIN4_NT;
    constexpr int NW = NT / 64;
    constexpr int KC = K - 4;                   // column bits of a group
    constexpr int NB = (1 << KC) / (32 * NW);   // 32-column blocks per wave
    constexpr int WB = __builtin_ctz(NW);       // column bits that name the wave
    constexpr int NG = FL_WIN4_MAX_GROUPS;
    constexpr int IT = (1 << (K - 1)) / NT;     // 16-byte tile accesses per thread and state
    static_assert(NB == 2 && (1 << KC) == 64 * NW, "a wave owns 64 columns");
    __shared__ __attribute__((aligned(16))) float2 lp[1 << K];
    __shared__ __attribute__((aligned(16))) float2 ll[1 << K];
    __shared__ float qacc[NG][512];
    const int h = pd.h;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int lc = lane & 31, lk = lane >> 5;
    for (int t = threadIdx.x; t < NG * 512; t += NT) (&qacc[0][0])[t] = 0.f;
    char* const pb = reinterpret_cast<char*>(lp);
    char* const lb = reinterpret_cast<char*>(ll);
    auto load_a = [&](int g, float (&dst)[16]) {
        const float4* M = mats + (size_t)g * 256 + (size_t)lane * 4;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const float4 t = M[q];
            dst[4 * q] = t.x;
            dst[4 * q + 1] = t.y;
            dst[4 * q + 2] = t.z;
            dst[4 * q + 3] = t.w;
        }
    };
    // tile element pairs (2 (tid + s NT), + 1) of both states, through
    // registers, so that the next tile's psi loads run under the current
    // tile's last group
    float4 tp[IT], tl[IT];
    auto fetch = [&](uint32_t tile, const float2* __restrict__ src, float4 (&dst)[IT]) {
        const uint64_t base = fl_tile_base(tile, C, W, h);
#pragma unroll
        for (int s = 0; s < IT; ++s)
            dst[s] = *reinterpret_cast<const float4*>(src + base + fl_tile_offset(2u * (threadIdx.x + s * NT), C, h));
    };
    auto put = [&]() {
#pragma unroll
        for (int s = 0; s < IT; ++s) {
            const uint32_t j = 2u * (threadIdx.x + s * NT);
            lp[fl_swz12(j)] = make_float2(tp[s].x, tp[s].y);
            lp[fl_swz12(j + 1)] = make_float2(tp[s].z, tp[s].w);
            ll[fl_swz12(j)] = make_float2(tl[s].x, tl[s].y);
            ll[fl_swz12(j + 1)] = make_float2(tl[s].z, tl[s].w);
        }
    };
    // the wave's columns are 64 w + (0 .. 63); which tile bits name the wave
    // depends only on how many of column bits KC - WB .. KC - 1 lie below u0
    auto part = [](int u) { return u <= KC - WB ? 0 : u - (KC - WB); };
    const float qsgn = (lc & 1) ? -1.0f : 1.0f;
    if (blockIdx.x < ntiles) {
        fetch(blockIdx.x, psi, tp);
        fetch(blockIdx.x, lam, tl);
        put();
    }
    for (uint32_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const uint32_t next = tile + gridDim.x;
        bool fetched = false;
        __syncthreads();
        float a[16], an[16];
        if (pd.ngroups > 0) load_a(0, a);
        for (int g = 0; g < pd.ngroups; ++g) {
            const int u0 = pass_u0(pd, g);
            load_a(g + 1 < pd.ngroups ? g + 1 : g, an);
            // (1) window overlap.  Step s takes columns 64 w + 2 s + k;
            // element spread(64 w + lk) | (lc >> 1) << u0 | spread(2 s)
            // (disjoint bits), component lc & 1: a per-lane byte offset XOR a
            // uniform one.
            const uint32_t ql = (fl_swz12(fl_spread((uint32_t)(64 * w + lk), u0, 4) | ((uint32_t)(lc >> 1) << u0)) * 8u) |
                                (4u * (uint32_t)(lc & 1));
            auto read_q = [&](int h0, float (&qx)[16], float (&qy)[16]) {
#pragma unroll
                for (int i = 0; i < 16; ++i) {
                    const int st = h0 + i;
                    const uint32_t o =
                        ql ^ __builtin_amdgcn_readfirstlane(fl_swz12(fl_spread((uint32_t)(2 * st), u0, 4)) * 8u);
                    qx[i] = *reinterpret_cast<const float*>(pb + o);
                    qy[i] = *reinterpret_cast<const float*>(lb + o);
                }
            };
            // (2) B operands of U^dagger on psi: amplitude 2t + lk of the
            // lane's column in block cb
            uint32_t vb[NB];
#pragma unroll
            for (int cb = 0; cb < NB; ++cb) vb[cb] = fl_swz12(fl_spread((uint32_t)(64 * w + 32 * cb + lc), u0, 4)) * 8u;
            const uint32_t lkoff = fl_swz12((uint32_t)lk << u0) * 8u;
            auto read_b = [&](const char* sb, float (&bq)[16][NB]) {
#pragma unroll
                for (int t = 0; t < 8; ++t) {
                    const uint32_t ss = fl_swz12((uint32_t)(2 * t) << u0) * 8u;
#pragma unroll
                    for (int cb = 0; cb < NB; ++cb) {
                        const float2 x = *reinterpret_cast<const float2*>(sb + ((vb[cb] ^ lkoff) ^ ss));
                        bq[t][cb] = x.x;
                        bq[t + 8][cb] = x.y;
                    }
                }
            };
            auto mfma_u = [&](const float (&bq)[16][NB], fl_f32x16 (&acc)[NB]) {
#pragma unroll
                for (int cb = 0; cb < NB; ++cb)
#pragma unroll
                    for (int r = 0; r < 16; ++r) acc[cb][r] = 0.0f;
#pragma unroll
                for (int st = 0; st < 16; ++st)
#pragma unroll
                    for (int cb = 0; cb < NB; ++cb)
                        acc[cb] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[st], bq[st][cb], acc[cb], 0, 0, 0);
            };
            // register r of block cb holds row 8 (r / 4) + 4 lk + r % 4 = 2 m + c
            auto write_u = [&](char* sb, const fl_f32x16 (&acc)[NB]) {
#pragma unroll
                for (int cb = 0; cb < NB; ++cb)
#pragma unroll
                    for (int q = 0; q < 4; ++q)
#pragma unroll
                        for (int p = 0; p < 2; ++p) {
                            const uint32_t m = 4 * q + 2 * lk + p;
                            float2 v;
                            v.x = acc[cb][4 * q + 2 * p];
                            v.y = acc[cb][4 * q + 2 * p + 1];
                            *reinterpret_cast<float2*>(sb + (vb[cb] ^ (fl_swz12(m << u0) * 8u))) = v;
                        }
            };
            // The phases in order, each one's LDS traffic placed between the
            // previous one's MFMAs (the scheduler pins 2 MFMAs : 1 LDS access):
            // Q reads A | Q MFMAs A + Q reads B | Q MFMAs B + psi reads |
            // Q sums | psi MFMAs + lambda reads | lambda MFMAs + psi writes |
            // lambda writes.  Each wave touches only its own columns, and its
            // LDS accesses run in program order.
            float bp[16][NB], bl[16][NB];
            fl_f32x16 ap[NB], al[NB];
            {
                fl_f32x16 dq;
#pragma unroll
                for (int r = 0; r < 16; ++r) dq[r] = 0.0f;
                float qa[16], qb[16], qc[16], qd[16];
                read_q(0, qa, qb);
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int i = 0; i < 16; ++i) dq = __builtin_amdgcn_mfma_f32_32x32x2f32(qa[i], qb[i], dq, 0, 0, 0);
                read_q(16, qc, qd);
#pragma unroll
                for (int i = 0; i < 16; ++i) {
                    __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);   // MFMA
                    __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);   // DS read
                }
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int i = 0; i < 16; ++i) dq = __builtin_amdgcn_mfma_f32_32x32x2f32(qc[i], qd[i], dq, 0, 0, 0);
                read_b(pb, bp);
#pragma unroll
                for (int i = 0; i < 16; ++i) {
                    __builtin_amdgcn_sched_group_barrier(0x008, 1, 1);   // MFMA
                    __builtin_amdgcn_sched_group_barrier(0x100, 1, 1);   // DS read
                }
                __builtin_amdgcn_sched_barrier(0);
                // register r of dq is row 8 (r / 4) + 4 lk + r % 4 of D; rows
                // (r, r + 1), r even, are window amplitude x = 4 (r / 4) + 2 lk +
                // (r % 4) / 2, components re, im, and this lane's column is
                // (y, b) = (lc >> 1, lc & 1).  With t = register r + 1 of the
                // neighbouring lane, b = 0 forms Re Q = D[2x][2y] + t and b = 1
                // forms Im Q = t - D[2x][2y+1].
#pragma unroll
                for (int pr = 0; pr < 8; ++pr) {
                    const int r = 2 * pr;
                    const float t = fl_dpp_f<0xB1>(dq[r + 1]);   // quad_perm(1,0,3,2): lane ^ 1
                    const float v = fmaf(qsgn, dq[r], t);
                    const int x = 4 * (pr >> 1) + 2 * lk + (pr & 1);
                    __hip_atomic_fetch_add(&qacc[g][(lc & 1) * 256 + 16 * x + (lc >> 1)], v, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_WORKGROUP);
                }
            }
            // the next tile's psi loads run under the last group's MFMAs
            if (g + 1 == pd.ngroups && next < ntiles) {
                fetch(next, psi, tp);
                fetched = true;
            }
            __builtin_amdgcn_sched_barrier(0);
            // (2) U^dagger on psi, with lambda's reads in between
            mfma_u(bp, ap);
            read_b(lb, bl);
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                __builtin_amdgcn_sched_group_barrier(0x008, 2, 2);   // MFMA
                __builtin_amdgcn_sched_group_barrier(0x100, 1, 2);   // DS read
            }
            __builtin_amdgcn_sched_barrier(0);
            // (3) U^dagger on lambda, with psi's writes in between
            mfma_u(bl, al);
            write_u(pb, ap);
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                __builtin_amdgcn_sched_group_barrier(0x008, 2, 3);   // MFMA
                __builtin_amdgcn_sched_group_barrier(0x200, 1, 3);   // DS write
            }
            __builtin_amdgcn_sched_barrier(0);
            write_u(lb, al);
            if (g + 1 == pd.ngroups || part(pass_u0(pd, g + 1)) != part(u0))
                __syncthreads();
            else
                __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (int k = 0; k < 16; ++k) a[k] = an[k];
        }
        const uint64_t base = fl_tile_base(tile, C, W, h);
        tile_store<float, K, NT, 1>(psi, base, K, C, h, lp);
        tile_store<float, K, NT, 1>(lam, base, K, C, h, ll);
        if (next < ntiles) {
            if (!fetched) fetch(next, psi, tp);
            fetch(next, lam, tl);
            __syncthreads();   // every wave has read the tile out of LDS
            put();
        }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < pd.ngroups * 512; t += NT)
        Qpart[(size_t)blockIdx.x * NG * 512 + t] = (double)(&qacc[0][0])[t];
}

// Qsum[t] += sum over the workgroups of Qpart[b][t] (t < nvals).  A block
// takes 32 consecutive values; its thread (v, j) sums rows b = j, j + 8, ...
// of value v (coalesced 256-byte rows), then the 8 partial sums of each value
// are added in j order, so the result does not depend on timing.
__global__ __launch_bounds__(256) void k_qsum(const double* __restrict__ Qpart, int nblocks, int nvals,
                                              double* __restrict__ Qsum) {
    __shared__ double part[8][32];
    const int v = threadIdx.x & 31, j = threadIdx.x >> 5;
    const int t = blockIdx.x * 32 + v;
    double s = 0.0;
    if (t < nvals) {
#pragma unroll 8
        for (int b = j; b < nblocks; b += 8) s += Qpart[(size_t)b * FL_WIN4_MAX_GROUPS * 512 + t];
    }
    part[j][v] = s;
    __syncthreads();
    if (j == 0 && t < nvals) {
        double r = part[0][v];
#pragma unroll
        for (int k = 1; k < 8; ++k) r += part[k][v];
        Qsum[t] += r;
    }
}

__global__ void k_zero(double* __restrict__ p, uint64_t n) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = 0.0;
}

// ---------------------------------------------------------------------------
// dense 6-qubit windows on the matrix cores (complex64 states)
// ---------------------------------------------------------------------------
// Every register group of a dense plan is one window of 6 consecutive tile
// bits [u0, u0+6); its gates were multiplied on the host (FP64) into a 64x64
// complex matrix U, applied here as the real 128x128 contraction
//   Y = A X,  A[2m'+c'][2m+c] = (Re U, -Im U; Im U, Re U)[c'][c] at (m', m),
// on the 128-column matrix X whose column v is the 64-vector of amplitudes
// sharing the other 7 tile bits, real index k = 2m + (0: re, 1: im).
// Wave w owns output rows [32w, 32w+32) and keeps its A rows in VGPRs.
//   MODE 0: FP32 MFMA v_mfma_f32_32x32x2f32 (k = 2 per step).
//   MODE 1: split BF16x3: X = Xh + Xl, A = Ah + Al (round-to-nearest-even
//           bf16 splits), Y = Ah Xh + Ah Xl + Al Xh with
//           v_mfma_f32_32x32x16_bf16 and FP32 accumulation.
// A fragments arrive pre-arranged per (wave, lane): MODE 0 as 64 floats
// (step kk = k/2), MODE 1 as 8 steps x 8 bf16 for hi, then the same for lo.


#define FL_DENSE_PLANE_STRIDE 136   // bf16 per column of a split plane (128 + 8 pad)

// FULL: the tile has the full KMAXD = 13 bits (every chain with L >= 13), so
// the column-block and element counts are compile-time constants.  The FP32
// tile uses the slots of fl_swz12: the 32 columns of a block read at one
// window position then meet at most two addresses per bank even for windows
// starting at bit 0, where fl_swz left them on 4 distinct slots.
template <int MODE, bool FULL>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_dense6(float2* __restrict__ psi, const float4* __restrict__ mats,
                                                uint32_t ntiles, int C, int W, fl_pass pd) {
    constexpr int KMAXD = 13;
    constexpr int TILE_BYTES = (1 << KMAXD) * 8;
    constexpr int PLANE_BYTES = 128 * FL_DENSE_PLANE_STRIDE * 2;
    constexpr int LDS_BYTES = (MODE == 1 && 2 * PLANE_BYTES > TILE_BYTES) ? 2 * PLANE_BYTES : TILE_BYTES;
    __shared__ __attribute__((aligned(16))) unsigned char smem[LDS_BYTES];
    float2* lds = reinterpret_cast<float2*>(smem);
    const int K = FULL ? KMAXD : C + W;
    const int h = pd.h;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int lc = lane & 31, lk = lane >> 5;
    const int ncb = FULL ? 4 : 1 << (K - 6 - 5);   // 32-column blocks (1, 2 or 4)
    const int ng = pd.ngroups;
    const uint64_t base = fl_tile_base(blockIdx.x, C, W, h);
    // full tiles: the unrolled form, every thread's 16 loads in flight at once
    if constexpr (FULL)
        tile_load<float, KMAXD, 256, 1>(psi, base, K, C, h, lds);
    else
        tile_load<float, 0, 256, 1>(psi, base, K, C, h, lds);
    __syncthreads();
    // write Y (registers of one window) back to the FP32 tile: register r of
    // block cb holds row 32w + 8(r/4) + 4 lk + r%4 (= 2m' + c'), column
    // 32 cb + lc; slot(cbase | m << u0) = slot(cbase) ^ slot(m << u0), the
    // second part uniform
    auto store_fp32 = [&](const fl_f32x16 (&acc)[4], const uint32_t (&cbase)[4], int u0) {
        const uint32_t mrow = 16 * w + 2 * lk;   // m of register 0 (rows 32w + 4lk, +1)
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
            if (cb < ncb) {
                const uint32_t vb = fl_swz12(cbase[cb]) * 8u;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
#pragma unroll
                    for (int p = 0; p < 2; ++p) {
                        const uint32_t m = mrow + 4 * q + p;   // rows 32w + 8q + 4lk + 2p, +1
                        float2 v;
                        v.x = acc[cb][4 * q + 2 * p];
                        v.y = acc[cb][4 * q + 2 * p + 1];
                        *reinterpret_cast<float2*>(smem + (vb ^ (fl_swz12(m << u0) * 8u))) = v;
                    }
                }
            }
        }
    };
    auto column_bases = [&](int u0, uint32_t (&cbase)[4]) {
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) cbase[cb] = fl_spread((32 * cb + lc) & ((1 << (K - 6)) - 1), u0, 6);
    };
    if constexpr (MODE == 0) {
        for (int g = 0; g < ng; ++g) {
            const int u0 = pass_u0(pd, g);
            // 4096 float4 (64 KiB) per window
            const float4* M = mats + (size_t)pass_gate(pd, g, 0) * 4096 + (size_t)(w * 64 + lane) * 16;
            uint32_t cbase[4];
            column_bases(u0, cbase);
            fl_f32x16 acc[4];
#pragma unroll
            for (int cb = 0; cb < 4; ++cb)
#pragma unroll
                for (int r = 0; r < 16; ++r) acc[cb][r] = 0.0f;
            float a[64];
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const float4 t = M[q];
                a[4 * q] = t.x;
                a[4 * q + 1] = t.y;
                a[4 * q + 2] = t.z;
                a[4 * q + 3] = t.w;
            }
            // element (column, m) of the tile sits at slot(cbase | m << u0) =
            // slot(cbase) ^ slot(m << u0) (the swizzle is linear over XOR); the
            // lane's half (re for lk = 0, im for lk = 1) is 4 lk bytes further
            uint32_t bb[4];
#pragma unroll
            for (int cb = 0; cb < 4; ++cb) bb[cb] = fl_swz12(cbase[cb]) * 8u + 4u * (uint32_t)lk;
            // B operands of step kk + 2 are read while step kk multiplies
            constexpr int PF = 2;
            float bq[PF + 1][4];
            auto fetch = [&](int kk, float (&dst)[4]) {
                const uint32_t sk = fl_swz12((uint32_t)kk << u0) * 8u;
#pragma unroll
                for (int cb = 0; cb < 4; ++cb)
                    if (cb < ncb) dst[cb] = *reinterpret_cast<const float*>(smem + (bb[cb] ^ sk));
            };
#pragma unroll
            for (int kk = 0; kk < PF; ++kk) fetch(kk, bq[kk]);
#pragma unroll
            for (int kk = 0; kk < 64; ++kk) {
                if (kk + PF < 64) fetch(kk + PF, bq[(kk + PF) % (PF + 1)]);
#pragma unroll
                for (int cb = 0; cb < 4; ++cb)
                    if (cb < ncb)
                        acc[cb] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[kk], bq[kk % (PF + 1)][cb], acc[cb], 0, 0, 0);
            }
            __syncthreads();
            store_fp32(acc, cbase, u0);
            __syncthreads();
        }
    } else {
        // The B operand of a window lives in LDS as two bf16 planes (hi, lo)
        // laid out [column][k]; element j of the tile (window bits from u) sits
        // at plane offset o_u(j) = col_u(j) STRIDE + 2 m_u(j) (+1 for the
        // imaginary part).  col_u and m_u are bit fields of j, so o_u is
        // additive over indices with disjoint bits.  The planes of the first
        // window come from the FP32 tile; those of every later window straight
        // from the previous window's accumulators (split once, when written),
        // and only the last window writes FP32 again, for the store.
        __bf16* ph = reinterpret_cast<__bf16*>(smem);
        __bf16* pl = ph + 128 * FL_DENSE_PLANE_STRIDE;
        typedef __bf16 bf2 __attribute__((ext_vector_type(2)));
        auto plane_off = [](uint32_t j, int u) {
            const uint32_t m = (j >> u) & 63;
            const uint32_t col = (j & ((1u << u) - 1)) | ((j >> (u + 6)) << u);
            return col * FL_DENSE_PLANE_STRIDE + 2 * m;
        };
        // (re, im) of one amplitude are adjacent in a plane: one 32-bit LDS
        // store per plane; hi = RNE_bf16(x), lo = RNE_bf16(x - hi)
        auto split_store = [&](float re, float im, uint32_t o) {
            bf2 hv, lv;
            hv.x = (__bf16)re;
            hv.y = (__bf16)im;
            lv.x = (__bf16)(re - (float)hv.x);
            lv.y = (__bf16)(im - (float)hv.y);
            *reinterpret_cast<bf2*>(ph + o) = hv;
            *reinterpret_cast<bf2*>(pl + o) = lv;
        };
        if (ng > 0) {
            // first window: every thread reads its amplitudes of the FP32
            // tile, the workgroup syncs, then the planes overwrite the tile
            constexpr int PER = (1 << KMAXD) / 256;
            float2 mine[PER];
            const int nper = FULL ? PER : (1 << K) / 256;
            const uint32_t l0 = fl_swz12(threadIdx.x);   // slot(tid + 256 t) = l0 ^ slot(256 t)
#pragma unroll
            for (int t = 0; t < PER; ++t)
                if (t < nper) mine[t] = lds[l0 ^ fl_swz12(256u * (uint32_t)t)];
            __syncthreads();
            const int u0 = pass_u0(pd, 0);
            const uint32_t otid = plane_off(threadIdx.x, u0);
#pragma unroll
            for (int t = 0; t < PER; ++t)
                if (t < nper)
                    // readfirstlane: keep the uniform term a scalar
                    split_store(mine[t].x, mine[t].y,
                                otid + __builtin_amdgcn_readfirstlane(plane_off(256u * (uint32_t)t, u0)));
            __syncthreads();
        }
        // A fragments of a window: 8 steps x 8 bf16 for hi, then for lo.  The
        // window stores each (Re, Im) pair of U once (32 KiB): lanes 2m' and
        // 2m'+1 of a half-wave load the same 16 bytes, and row 2m' takes them
        // as (Re, -Im), row 2m'+1 as (Im, Re): a rotation by 16 bits per lane
        // parity, then a sign flip of the high half for the even rows.
        fl_bf16x8 ah[8], al[8];
        const uint32_t rot = 16u * (uint32_t)(lane & 1);
        const uint32_t neg = (lane & 1) ? 0u : 0x80000000u;
        auto fix = [&](const float4& t) {
            uint4 u = *reinterpret_cast<const uint4*>(&t);
            u.x = __builtin_amdgcn_alignbit(u.x, u.x, rot) ^ neg;
            u.y = __builtin_amdgcn_alignbit(u.y, u.y, rot) ^ neg;
            u.z = __builtin_amdgcn_alignbit(u.z, u.z, rot) ^ neg;
            u.w = __builtin_amdgcn_alignbit(u.w, u.w, rot) ^ neg;
            return *reinterpret_cast<const fl_bf16x8*>(&u);
        };
        auto load_a = [&](int g) {
            const float4* M = mats + (size_t)pass_gate(pd, g, 0) * 2048 + (size_t)(w * 16 * 16 + lk * 16 + (lc >> 1));
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const float4 th = M[q * 32], tl = M[1024 + q * 32];
                ah[q] = fix(th);
                al[q] = fix(tl);
            }
        };
        if (ng > 0) load_a(0);
        for (int g = 0; g < ng; ++g) {
            const int u0 = pass_u0(pd, g);
            uint32_t cbase[4];
            column_bases(u0, cbase);
            fl_f32x16 acc[4];
#pragma unroll
            for (int cb = 0; cb < 4; ++cb)
#pragma unroll
                for (int r = 0; r < 16; ++r) acc[cb][r] = 0.0f;
#pragma unroll
            for (int st = 0; st < 8; ++st) {
                const int k0 = 16 * st + 8 * lk;
#pragma unroll
                for (int cb = 0; cb < 4; ++cb) {
                    if (cb < ncb) {
                        const uint32_t col = 32 * cb + lc;
                        const uint32_t o = col * FL_DENSE_PLANE_STRIDE + k0;
                        const fl_bf16x8 bh = *reinterpret_cast<const fl_bf16x8*>(ph + o);
                        const fl_bf16x8 bl = *reinterpret_cast<const fl_bf16x8*>(pl + o);
                        acc[cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[st], bh, acc[cb], 0, 0, 0);
                        acc[cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[st], bl, acc[cb], 0, 0, 0);
                        acc[cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[st], bh, acc[cb], 0, 0, 0);
                    }
                }
            }
            // the next window's fragments go into the registers just freed,
            // so that their latency overlaps the barrier and the split
            if (g + 1 < ng) load_a(g + 1);
            __syncthreads();   // every wave has read this window's planes
            if (g + 1 < ng) {
                // element of register (cb, q, p): j = cbase[cb] | (mrow + 4q + p) << u0,
                // three parts with disjoint bits: o(j) = o(cbase | mrow << u0) + o((4q + p) << u0)
                const int un = pass_u0(pd, g + 1);
                const uint32_t mrow = 16 * w + 2 * lk;
#pragma unroll
                for (int cb = 0; cb < 4; ++cb) {
                    if (cb < ncb) {
                        const uint32_t ob = plane_off(cbase[cb] | (mrow << u0), un);
#pragma unroll
                        for (int q = 0; q < 4; ++q)
#pragma unroll
                            for (int p = 0; p < 2; ++p)
                                split_store(acc[cb][4 * q + 2 * p], acc[cb][4 * q + 2 * p + 1],
                                            ob + __builtin_amdgcn_readfirstlane(
                                                     plane_off((uint32_t)(4 * q + p) << u0, un)));
                    }
                }
            } else {
                store_fp32(acc, cbase, u0);
            }
            __syncthreads();
        }
    }
    if constexpr (FULL)
        tile_store<float, KMAXD, 256, 1>(psi, base, K, C, h, lds);
    else
        tile_store<float, 0, 256, 1>(psi, base, K, C, h, lds);
}

// ---------------------------------------------------------------------------
// dense 4-qubit windows on the FP32 matrix cores (complex64 states)
// ---------------------------------------------------------------------------
// Every register group of a dense-4 plan is one window of 4 consecutive tile
// bits [u0, u0+4); its gates were multiplied on the host (FP64) into a 16x16
// complex matrix U, applied as the real 32x32 contraction Y = A X with
// A[2m'+c'][2m+c] = (Re U, -Im U; Im U, Re U)[c'][c] at (m', m): exactly one
// v_mfma_f32_32x32x2f32 output tile, K = 32 in 16 steps of 2.  Column v of X
// is the 16-vector of amplitudes sharing the other 9 tile bits; a tile has
// 512 columns, 512 / NW per wave (blocks of 32).  The contraction index runs
// component-major, k' = 16 c + m: step s takes k' = 2s + l/32, so lane l
// supplies A[l%32][k'] (16 VGPRs, the same for every wave) and, per block,
// component s/8 of amplitude 2(s mod 8) + l/32 of its column; steps s and
// s + 8 use the two halves of one 8-byte LDS read.  A wave reads and writes
// only its own columns: the columns of wave w are those whose log2(NW)
// highest bits outside the window equal w, so consecutive windows that leave
// the same tile bits to the wave index (with NW = 8 all windows below bit 7
// leave bits 10, 11 and 12) need no barrier between them, only this wave's
// own LDS order.
template <int NW>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(NW / 2))) void k_dense4(
    float2* __restrict__ psi, const float4* __restrict__ mats, int W, fl_pass pd) {
    constexpr int K = 13;
    constexpr int C = FL_DENSE4_LOWBITS;
    constexpr int NB = 16 / NW;                  // 32-column blocks per wave (512 columns per tile)
    constexpr int WB = __builtin_ctz(NW);        // column bits that name the wave
    __shared__ __attribute__((aligned(16))) float2 lds[1 << K];
    const char* const lbytes = reinterpret_cast<const char*>(lds);
    const int h = pd.h;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int lc = lane & 31, lk = lane >> 5;
    const uint64_t base = fl_tile_base(blockIdx.x, C, W, h);
    tile_load<float, K, 64 * NW>(psi, base, K, C, h, lds);
    __syncthreads();
    // A fragments of a window: 64 lanes x 16 floats (4 KiB).  The next
    // window's fragments are fetched while the current window is applied; the
    // last window fetches its own again, so that no branch lets the loads
    // drift down to their use.
    auto load_a = [&](int g, float (&dst)[16]) {
        const float4* M = mats + (size_t)pass_gate(pd, g, 0) * 256 + (size_t)lane * 4;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const float4 t = M[q];
            dst[4 * q] = t.x;
            dst[4 * q + 1] = t.y;
            dst[4 * q + 2] = t.z;
            dst[4 * q + 3] = t.w;
        }
    };
    float a[16], an[16];
    if (pd.ngroups > 0) load_a(0, a);
    for (int g = 0; g < pd.ngroups; ++g) {
        const int u0 = pass_u0(pd, g);
        load_a(g + 1 < pd.ngroups ? g + 1 : g, an);
        __builtin_amdgcn_sched_barrier(0);
        // slot(spread(col) | s << u0) = slot(spread(col)) ^ slot(s << u0): the
        // second part is uniform (the swizzle is linear over XOR)
        uint32_t vb[NB];
#pragma unroll
        for (int cb = 0; cb < NB; ++cb)
            vb[cb] = fl_swz(fl_spread((uint32_t)(32 * NB * w + 32 * cb + lc), u0, 4)) * 8u;
        fl_f32x16 acc[NB];
#pragma unroll
        for (int cb = 0; cb < NB; ++cb)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[cb][r] = 0.0f;
        float bq[16][NB];
        // amplitude 2t + lk of the column: slot(spread(col)) ^ slot(lk << u0) ^ slot(2t << u0)
        const uint32_t lkoff = fl_swz((uint32_t)lk << u0) * 8u;
        auto read_b = [&](int cb) {
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                const uint32_t ss = fl_swz((uint32_t)(2 * t) << u0) * 8u;
                const float2 x = *reinterpret_cast<const float2*>(lbytes + ((vb[cb] ^ lkoff) ^ ss));
                bq[t][cb] = x.x;
                bq[t + 8][cb] = x.y;
            }
        };
        auto mfma_b = [&](int cb) {
#pragma unroll
            for (int st = 0; st < 16; ++st)
                acc[cb] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[st], bq[st][cb], acc[cb], 0, 0, 0);
        };
        // register r of block cb holds row 8(r/4) + 4 lk + r%4 = 2m' + c'
        auto write_b = [&](int cb) {
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int p = 0; p < 2; ++p) {
                    const uint32_t m = 4 * q + 2 * lk + p;
                    float2 v;
                    v.x = acc[cb][4 * q + 2 * p];
                    v.y = acc[cb][4 * q + 2 * p + 1];
                    *reinterpret_cast<float2*>(reinterpret_cast<char*>(lds) + (vb[cb] ^ (fl_swz(m << u0) * 8u))) = v;
                }
        };
        // Blocks in two halves, so that the LDS traffic of one half runs
        // under the MFMAs of the other: read the first half, then its MFMAs
        // with the second half's reads in between, then the second half's
        // MFMAs with the first half's writes in between, then those writes.
        // (Each block reads and writes only its own columns.)
        constexpr int HB = NB / 2;
#pragma unroll
        for (int cb = 0; cb < HB; ++cb) read_b(cb);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int cb = 0; cb < HB; ++cb) mfma_b(cb);
#pragma unroll
        for (int cb = HB; cb < NB; ++cb) read_b(cb);
#pragma unroll
        for (int i = 0; i < 8 * HB; ++i) {
            __builtin_amdgcn_sched_group_barrier(0x008, 2, 0);   // MFMA
            __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);   // DS read
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int cb = HB; cb < NB; ++cb) mfma_b(cb);
#pragma unroll
        for (int cb = 0; cb < HB; ++cb) write_b(cb);
#pragma unroll
        for (int i = 0; i < 8 * HB; ++i) {
            __builtin_amdgcn_sched_group_barrier(0x008, 2, 1);   // MFMA
            __builtin_amdgcn_sched_group_barrier(0x200, 1, 1);   // DS write
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int cb = HB; cb < NB; ++cb) write_b(cb);
        // the WB tile bits that select a wave's columns: column bits 9 - WB .. 8,
        // which sit 4 higher when at or above the window, so the set depends
        // only on how many of them lie below u0
        auto part = [](int u) { return u <= 9 - WB ? 0 : u - (9 - WB); };
        if (g + 1 == pd.ngroups || part(pass_u0(pd, g + 1)) != part(u0))
            __syncthreads();
        else
            __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int k = 0; k < 16; ++k) a[k] = an[k];
    }
    tile_store<float, K, 64 * NW>(psi, base, K, C, h, lds);
}

// ---------------------------------------------------------------------------
// launch wrappers
// ---------------------------------------------------------------------------

static inline uint32_t ntiles_of(const fl_geom& g) { return 1u << (g.L - g.K); }

hipError_t launch_sweep(int dtype, const fl_geom& g, void* psi, const void* gates, const fl_pass& pd,
                        hipStream_t s) {
    const dim3 grid(ntiles_of(g)), block(FL_NT);
    if (dtype == 0) {
        float2* p = (float2*)psi;
        const float* G = (const float*)gates;
        if (g.K == FL_KMAX_C64 && g.W > 0) {
            if (g.C != FL_SWEEP_LOWBITS_C64) return hipErrorInvalidValue;
            if (2 * (g.L - 1) > FL_MAX_GATE_TABLE) return hipErrorInvalidValue;
            hipLaunchKernelGGL(
                (k_sweep_tiles<float, FL_SWEEP_R_C64, FL_KMAX_C64, FL_SWEEP_NT_C64, FL_SWEEP_LOWBITS_C64, FL_SWEEP_LDS_GATES != 0>), grid,
                dim3(FL_SWEEP_NT_C64), 0, s, p, G, g.W, pd, 2 * (g.L - 1));
        } else if (g.R == 5)
            hipLaunchKernelGGL((k_sweep<float, 5, 0, FL_KMAX_C64>), grid, block, 0, s, p, G, g.C, g.W, pd);
        else if (g.R == 4)
            hipLaunchKernelGGL((k_sweep<float, 4, 0, FL_KMAX_C64>), grid, block, 0, s, p, G, g.C, g.W, pd);
        else if (g.R == 3)
            hipLaunchKernelGGL((k_sweep<float, 3, 0, FL_KMAX_C64>), grid, block, 0, s, p, G, g.C, g.W, pd);
        else
            hipLaunchKernelGGL((k_sweep<float, 2, 0, FL_KMAX_C64>), grid, block, 0, s, p, G, g.C, g.W, pd);
    } else {
        double2* p = (double2*)psi;
        const double* G = (const double*)gates;
        if (g.K == FL_KMAX_C128 && g.W > 0) {
            if (g.C != FL_LOWBITS) return hipErrorInvalidValue;
            hipLaunchKernelGGL((k_sweep_tiles<double, 4, FL_KMAX_C128, 256, FL_LOWBITS, false>), grid, dim3(256), 0, s,
                               p, G, g.W, pd, 0);
        } else if (g.R == 4)
            hipLaunchKernelGGL((k_sweep<double, 4, 0, FL_KMAX_C128>), grid, block, 0, s, p, G, g.C, g.W, pd);
        else if (g.R == 3)
            hipLaunchKernelGGL((k_sweep<double, 3, 0, FL_KMAX_C128>), grid, block, 0, s, p, G, g.C, g.W, pd);
        else
            hipLaunchKernelGGL((k_sweep<double, 2, 0, FL_KMAX_C128>), grid, block, 0, s, p, G, g.C, g.W, pd);
    }
    return hipGetLastError();
}

hipError_t launch_rdm(int dtype, const fl_geom& g, const void* psi, const fl_pass& pd, double* partials, int grid,
                      int nslot, hipStream_t s) {
    const uint32_t nt = ntiles_of(g);
    if (dtype == 0) {
        const float2* p = (const float2*)psi;
        if (g.K == FL_KMAX_RDM && g.W > 0)
            hipLaunchKernelGGL((k_rdm_tiles<float, FL_KMAX_RDM, 256>), dim3(grid), dim3(256), 0, s, p, g.W, nt, pd,
                               partials, nslot);
        else
            hipLaunchKernelGGL((k_rdm<float, 0, FL_KMAX_RDM>), dim3(grid), dim3(FL_NT), 0, s, p, g.C, g.W, nt, pd,
                               partials, nslot);
    } else {
        const double2* p = (const double2*)psi;
        if (g.K == FL_KMAX_RDM && g.W > 0)
            hipLaunchKernelGGL((k_rdm_tiles<double, FL_KMAX_RDM, 256>), dim3(grid), dim3(256), 0, s, p, g.W, nt, pd,
                               partials, nslot);
        else
            hipLaunchKernelGGL((k_rdm<double, 0, FL_KMAX_RDM>), dim3(grid), dim3(FL_NT), 0, s, p, g.C, g.W, nt, pd,
                               partials, nslot);
    }
    return hipGetLastError();
}

hipError_t launch_rdm_groups(const fl_geom& g, const void* psi, const fl_pass& pd, double* partials, int grid,
                             int nslot, hipStream_t s) {
    if (g.K != FL_KMAX_C64 || g.R != FL_RDM_R_C64 || g.W == 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_rdm_groups<FL_RDM_R_C64, FL_KMAX_C64, FL_RDM_NT_C64>), dim3(grid), dim3(FL_RDM_NT_C64), 0,
                       s, (const float2*)psi, g.W, ntiles_of(g), pd, partials, nslot);
    return hipGetLastError();
}

hipError_t launch_energy_contract(const double* red, const double* h64, int L, double* out, double* rdm, hipStream_t s) {
    if (L < 2 || L > 65) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_energy_contract, dim3(1), dim3(64), 0, s, red, h64, L, out, rdm);
    return hipGetLastError();
}

hipError_t launch_finalize(const double* partials, int nblocks, int nvals, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_finalize, dim3(nvals), dim3(256), 0, s, partials, nblocks, nvals, out);
    return hipGetLastError();
}

hipError_t launch_init(int dtype, void* psi, int L, const void* tabs, int a, int b, hipStream_t s) {
    const uint64_t n = 1ull << L;
    const double2* t = (const double2*)tabs;
    const double2* tlo = t;
    const double2* tmid = t + (1 << a);
    const double2* thi = tmid + (1 << b);
    const uint64_t want = (n + 255) / 256;
    const unsigned grid = (unsigned)(want < 65536 ? want : 65536);
    if (dtype == 0 && a >= 1) {
        const uint64_t want2 = (n / 2 + 255) / 256;
        hipLaunchKernelGGL(k_init_pairs_c64, dim3((unsigned)(want2 < 65536 ? want2 : 65536)), dim3(256), 0, s,
                           (float4*)psi, tlo, tmid, thi, a, b, n / 2);
    } else if (dtype == 0)
        hipLaunchKernelGGL(k_init<float>, dim3(grid), dim3(256), 0, s, (float2*)psi, tlo, tmid, thi, a, b, n);
    else
        hipLaunchKernelGGL(k_init<double>, dim3(grid), dim3(256), 0, s, (double2*)psi, tlo, tmid, thi, a, b, n);
    return hipGetLastError();
}

hipError_t launch_overlap(int dta, const void* a, int dtb, const void* b, uint64_t n, double* partials, int grid,
                          hipStream_t s) {
    if (dta == 1 && dtb == 0)
        hipLaunchKernelGGL((k_overlap<double, float>), dim3(grid), dim3(256), 0, s, (const double2*)a, (const float2*)b,
                           n, partials);
    else if (dta == 1 && dtb == 1)
        hipLaunchKernelGGL((k_overlap<double, double>), dim3(grid), dim3(256), 0, s, (const double2*)a,
                           (const double2*)b, n, partials);
    else if (dta == 0 && dtb == 1)
        hipLaunchKernelGGL((k_overlap<float, double>), dim3(grid), dim3(256), 0, s, (const float2*)a,
                           (const double2*)b, n, partials);
    else
        hipLaunchKernelGGL((k_overlap<float, float>), dim3(grid), dim3(256), 0, s, (const float2*)a, (const float2*)b,
                           n, partials);
    return hipGetLastError();
}

hipError_t launch_apply_h(int dtype, const fl_geom& g, const void* psi, void* lam, const void* hmat, const fl_pass& pd,
                          int first, hipStream_t s) {
    const dim3 grid(ntiles_of(g)), block(FL_NT);
    if (dtype == 0) {
        if (g.K == FL_KMAX_C64)
            hipLaunchKernelGGL((k_apply_h<float, FL_KMAX_C64, FL_KMAX_C64>), grid, block, 0, s, (const float2*)psi,
                               (float2*)lam, (const float*)hmat, g.C, g.W, pd, first);
        else
            hipLaunchKernelGGL((k_apply_h<float, 0, FL_KMAX_C64>), grid, block, 0, s, (const float2*)psi,
                               (float2*)lam, (const float*)hmat, g.C, g.W, pd, first);
    } else {
        if (g.K == FL_KMAX_C128)
            hipLaunchKernelGGL((k_apply_h<double, FL_KMAX_C128, FL_KMAX_C128>), grid, block, 0, s,
                               (const double2*)psi, (double2*)lam, (const double*)hmat, g.C, g.W, pd, first);
        else
            hipLaunchKernelGGL((k_apply_h<double, 0, FL_KMAX_C128>), grid, block, 0, s, (const double2*)psi,
                               (double2*)lam, (const double*)hmat, g.C, g.W, pd, first);
    }
    return hipGetLastError();
}

hipError_t launch_adjoint(int dtype, const fl_geom& g, void* psi, void* lam, const void* gates, const fl_pass& pd,
                          double* Mpart, int grid, hipStream_t s) {
    const uint32_t nt = ntiles_of(g);
    const int nb = g.L - 1;
    if (dtype == 0) {
        float2* p = (float2*)psi;
        float2* l = (float2*)lam;
        const float* G = (const float*)gates;
        if (g.K == FL_KMAX_ADJ && g.R == 4)
            hipLaunchKernelGGL((k_adjoint<float, 4, FL_KMAX_ADJ, FL_KMAX_ADJ>), dim3(grid), dim3(FL_NT), 0, s, p, l, G,
                               g.C, g.W, nt, pd, Mpart, nb);
        else if (g.R == 4)
            hipLaunchKernelGGL((k_adjoint<float, 4, 0, FL_KMAX_ADJ>), dim3(grid), dim3(FL_NT), 0, s, p, l, G, g.C, g.W,
                               nt, pd, Mpart, nb);
        else if (g.R == 3)
            hipLaunchKernelGGL((k_adjoint<float, 3, 0, FL_KMAX_ADJ>), dim3(grid), dim3(FL_NT), 0, s, p, l, G, g.C, g.W,
                               nt, pd, Mpart, nb);
        else
            hipLaunchKernelGGL((k_adjoint<float, 2, 0, FL_KMAX_ADJ>), dim3(grid), dim3(FL_NT), 0, s, p, l, G, g.C, g.W,
                               nt, pd, Mpart, nb);
    } else {
        double2* p = (double2*)psi;
        double2* l = (double2*)lam;
        const double* G = (const double*)gates;
        if (g.K == FL_KMAX_ADJ && g.R == 4)
            hipLaunchKernelGGL((k_adjoint<double, 4, FL_KMAX_ADJ, FL_KMAX_ADJ>), dim3(grid), dim3(FL_NT), 0, s, p, l,
                               G, g.C, g.W, nt, pd, Mpart, nb);
        else if (g.R == 4)
            hipLaunchKernelGGL((k_adjoint<double, 4, 0, FL_KMAX_ADJ>), dim3(grid), dim3(FL_NT), 0, s, p, l, G, g.C,
                               g.W, nt, pd, Mpart, nb);
        else if (g.R == 3)
            hipLaunchKernelGGL((k_adjoint<double, 3, 0, FL_KMAX_ADJ>), dim3(grid), dim3(FL_NT), 0, s, p, l, G, g.C,
                               g.W, nt, pd, Mpart, nb);
        else
            hipLaunchKernelGGL((k_adjoint<double, 2, 0, FL_KMAX_ADJ>), dim3(grid), dim3(FL_NT), 0, s, p, l, G, g.C,
                               g.W, nt, pd, Mpart, nb);
    }
    return hipGetLastError();
}

hipError_t launch_adjoint_win4(const fl_geom& g, void* psi, void* lam, const void* mats, const fl_pass& pd,
                               double* Qpart, int grid, double* Qsum, hipStream_t s) {
    if (g.K != FL_KMAX_C64 || g.R != 4 || g.C != FL_DENSE4_LOWBITS || g.C + g.W != FL_KMAX_C64 ||
        pd.ngroups > FL_WIN4_MAX_GROUPS || grid < 1)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_adjoint_win4, dim3(grid), dim3(FL_WIN4_NT), 0, s, (float2*)psi, (float2*)lam,
                       (const float4*)mats, g.W, ntiles_of(g), pd, Qpart);
    const int nvals = pd.ngroups * 512;
    if (nvals > 0) hipLaunchKernelGGL(k_qsum, dim3((nvals + 31) / 32), dim3(256), 0, s, Qpart, grid, nvals, Qsum);
    return hipGetLastError();
}

hipError_t launch_zero(double* p, uint64_t n, hipStream_t s) {
    const uint64_t want = (n + 255) / 256;
    const unsigned grid = (unsigned)(want < 4096 ? (want ? want : 1) : 4096);
    hipLaunchKernelGGL(k_zero, dim3(grid), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_dense4(const fl_geom& g, void* psi, const void* mats, const fl_pass& pd, hipStream_t s) {
    if (g.C + g.W != 13) return hipErrorInvalidValue;
    if (g.W == 0) {
        // a single 13-bit tile (L = 13): the same amplitudes as low bits
        // [0, C) plus the window [C, 13), the kernel's fixed geometry
        fl_pass p = pd;
        p.h = FL_DENSE4_LOWBITS;
        hipLaunchKernelGGL(k_dense4<FL_DENSE4_NW>, dim3(1), dim3(64 * FL_DENSE4_NW), 0, s, (float2*)psi,
                           (const float4*)mats, 13 - FL_DENSE4_LOWBITS, p);
        return hipGetLastError();
    }
    if (g.C != FL_DENSE4_LOWBITS) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_dense4<FL_DENSE4_NW>, dim3(ntiles_of(g)), dim3(64 * FL_DENSE4_NW), 0, s, (float2*)psi,
                       (const float4*)mats, g.W, pd);
    return hipGetLastError();
}

hipError_t launch_dense6(int mode, const fl_geom& g, void* psi, const void* mats, const fl_pass& pd, hipStream_t s) {
    const uint32_t nt = ntiles_of(g);
    const bool full = g.C + g.W == 13;
    if (mode == 0 && full)
        hipLaunchKernelGGL((k_dense6<0, true>), dim3(nt), dim3(256), 0, s, (float2*)psi, (const float4*)mats, nt, g.C,
                           g.W, pd);
    else if (mode == 0)
        hipLaunchKernelGGL((k_dense6<0, false>), dim3(nt), dim3(256), 0, s, (float2*)psi, (const float4*)mats, nt, g.C,
                           g.W, pd);
    else if (full)
        hipLaunchKernelGGL((k_dense6<1, true>), dim3(nt), dim3(256), 0, s, (float2*)psi, (const float4*)mats, nt, g.C,
                           g.W, pd);
    else
        hipLaunchKernelGGL((k_dense6<1, false>), dim3(nt), dim3(256), 0, s, (float2*)psi, (const float4*)mats, nt, g.C,
                           g.W, pd);
    return hipGetLastError();
}

}  // namespace fl
