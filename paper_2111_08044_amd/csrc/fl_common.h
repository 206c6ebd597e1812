// Shared definitions of the Floquet brickwork engine: tile geometry, pass
// descriptors and the index maps used by both the host planner and the HIP
// kernels.
//
// State layout in HBM: one contiguous array of 2^L interleaved complex
// amplitudes (re, im), complex64 or complex128.  Amplitude index
// x = sum_j bit_j 2^(L-1-j): site 0 is the most significant bit, matching the
// wavefunction psi_{b1...bL} with b1 leading (Sec. II).  Bond b joins sites
// (b, b+1) and therefore the two bits p = L-2-b and p+1; the 4x4 gate acts on
// the local index 2*bit(p+1) + bit(p).
//
// A "pass" streams the whole state through the chip once.  The amplitudes are
// split into tiles of 2^K that share every bit outside a tile bit set
// S = [0, C) u [h, h+W) (K = C + W); the C low bits keep every tile made of
// 2^W contiguous runs of 2^C amplitudes, so loads and stores coalesce.  Inside
// the tile, tile-local bit u maps to physical bit u (u < C) or h + u - C.
// A pass applies an ordered list of "groups"; a group names R consecutive
// tile-local bits [u0, u0+R) that each thread holds in registers (2^R
// amplitudes) while it applies the group's ops, each op a 4x4 gate on the
// register bits (i, i+1), optionally preceded by a reduction into a slot.
#pragma once
#include <stddef.h>
#include <stdint.h>

#if defined(__HIPCC__)
#define FL_HD __host__ __device__ inline
#else
#define FL_HD inline
#endif

#define FL_NT 256            // threads per workgroup of the tile kernels
#define FL_MAX_GROUPS 40     // groups per pass
#define FL_MAX_OPS 12        // ops per group
#define FL_LOWBITS 6         // C for chains longer than one tile
#define FL_KMAX_C64 13       // tile bits for complex64 (64 KiB of LDS)
#define FL_KMAX_C128 12      // tile bits for complex128 (64 KiB of LDS)
#define FL_KMAX_ADJ 12       // tile bits of the two-state adjoint pass (complex64)
#define FL_WIN4_MAX_GROUPS 14  // register groups per pass of a 4-qubit-window plan (the reverse pass keeps one window-overlap sum per group)
#define FL_WIN4_NT 512         // threads of the 4-qubit-window reverse pass (13-bit tiles of two states)
#define FL_KMAX_RDM 12       // tile bits of the energy / density-matrix reduction
#define FL_MAX_SLOTS 16      // distinct reduction slots per pass
#define FL_MAX_GATE_TABLE 66 // gates of the largest chain (L = 34): G_b and G_b^dagger per bond
#ifndef FL_SWEEP_NT_C64
#define FL_SWEEP_NT_C64 512  // threads per workgroup of the complex64 full-tile sweep
#endif
#ifndef FL_SWEEP_LOWBITS_C64
#define FL_SWEEP_LOWBITS_C64 4  // C of the complex64 sweep: 16-amplitude (128-byte) runs, a 9-bit window
#endif
#ifndef FL_SWEEP_R_C64
#define FL_SWEEP_R_C64 4     // register bits per group of the complex64 sweep
#endif
#ifndef FL_SWEEP_LDS_GATES
#define FL_SWEEP_LDS_GATES 1  // complex64 sweep: gates in vector registers, read from an LDS copy of the table
#endif
#define FL_RDM_NT_C64 256    // threads per workgroup of the complex64 bond reduction on 13-bit tiles
#define FL_RDM_R_C64 5       // register bits per group of that reduction
#ifndef FL_RDM_GROUPS
#define FL_RDM_GROUPS 1      // complex64 reductions on 13-bit tiles with register groups (L >= 14)
#endif
#ifndef FL_DENSE4_LOWBITS
#define FL_DENSE4_LOWBITS 4  // C of the 4-qubit-window form (forward and reverse pass)
#endif
#ifndef FL_DENSE4_NW
#define FL_DENSE4_NW 4       // waves per workgroup of the 4-qubit-window MFMA kernel
#endif
#ifndef FL_DIRECT_MIN_U0
#define FL_DIRECT_MIN_U0 4   // lowest group bit for direct HBM <-> register transfers
#endif

struct fl_pass {
    int32_t h;                               // first physical bit of the high window
    int32_t ngroups;
    int32_t flags;                           // kernel-specific (e.g. "also reduce the norm")
    int32_t nslots;                          // distinct reduction slots used by the ops
    int8_t sbond[FL_MAX_SLOTS];              // bond of each slot
    int8_t u0[FL_MAX_GROUPS];                // first tile-local register bit of each group
    int8_t nops[FL_MAX_GROUPS];
    int8_t opi[FL_MAX_GROUPS][FL_MAX_OPS];   // op acts on register bits (i, i+1)
    int16_t opg[FL_MAX_GROUPS][FL_MAX_OPS];  // gate-table index, -1 = no gate
    int16_t ops[FL_MAX_GROUPS][FL_MAX_OPS];  // reduction slot (index into sbond), -1 = none
};

#ifdef __cplusplus
// Kernels read the per-op arrays as aligned 32-bit words (scalar loads).
static_assert(offsetof(fl_pass, u0) % 4 == 0 && sizeof(((fl_pass*)0)->u0) % 4 == 0, "u0 not word aligned");
static_assert(offsetof(fl_pass, nops) % 4 == 0 && sizeof(((fl_pass*)0)->nops) % 4 == 0, "nops not word aligned");
static_assert(offsetof(fl_pass, opi) % 4 == 0 && sizeof(((fl_pass*)0)->opi[0]) % 4 == 0, "opi rows not word aligned");
static_assert(offsetof(fl_pass, opg) % 4 == 0 && sizeof(((fl_pass*)0)->opg[0]) % 4 == 0, "opg rows not word aligned");
static_assert(offsetof(fl_pass, ops) % 4 == 0 && sizeof(((fl_pass*)0)->ops[0]) % 4 == 0, "ops rows not word aligned");
#endif

struct fl_geom {
    int L, C, W, K, R;
};

// Offset of the first amplitude of tile `tile` for window start h.
FL_HD uint64_t fl_tile_base(uint64_t tile, int C, int W, int h) {
    const int nmid = h - C;
    const uint64_t mid = tile & ((1ull << nmid) - 1ull);
    const uint64_t top = tile >> nmid;
    return (mid << C) | (top << (h + W));
}

// Offset, relative to the tile base, of tile-local amplitude j.
FL_HD uint64_t fl_tile_offset(uint32_t j, int C, int h) {
    return (uint64_t)(j & ((1u << C) - 1u)) | ((uint64_t)(j >> C) << h);
}

// LDS slot of tile-local amplitude j.  XOR-ing bits 4..7 into bits 0..3
// makes the access patterns of 4-bit register groups (any first bit u0) and
// of pairwise tile loads hit 16 distinct 8-byte slots within each run of 16
// lanes.  The function is linear over XOR: slot(a ^ b) = slot(a) ^ slot(b).
FL_HD uint32_t fl_swz(uint32_t j) { return j ^ ((j >> 4) & 15u); }

// The same folding of bits 8..11 as well (also linear over XOR): 16 lanes
// that step through a 4-bit window's amplitudes at stride 2^u0 then hit 16
// distinct 8-byte slots for every u0 of a 12-bit tile (and meet at most two
// addresses per bank on 13-bit tiles), as do the column and pairwise patterns
// fl_swz serves.  The window form's reverse pass reads its tiles both ways.
FL_HD uint32_t fl_swz12(uint32_t j) { return j ^ ((j >> 4) & 15u) ^ ((j >> 8) & 15u); }

// Insert R zero bits at position u0 into o.
FL_HD uint32_t fl_spread(uint32_t o, int u0, int R) {
    const uint32_t lo = o & ((1u << u0) - 1u);
    return lo | ((o >> u0) << (u0 + R));
}

// Tile-local bit of physical bit p for window start h (-1 if p is not in S).
FL_HD int fl_local_bit(int p, int C, int W, int h) {
    if (p < C) return p;
    if (p >= h && p < h + W) return C + (p - h);
    return -1;
}
