// Fusion planner: turns n periods of the brickwork circuit into tile passes.
#pragma once
#include <vector>

#include "fl_common.h"

namespace fl {

// Tile geometry for a chain of L sites; kmax = tile bits, r = register bits,
// lowbits = C, the contiguous low bits of every tile when L > kmax.  A smaller
// C leaves a wider window of high bits, which the brickwork's light cones
// cross in fewer passes; C = 4 still keeps every run of a tile one 128-byte
// line of complex64 amplitudes.
fl_geom make_geom(int L, int kmax, int r, int lowbits = FL_LOWBITS);

struct PlanStats {
    long long passes = 0;
    long long gates = 0;
    long long groups = 0;
};

// Passes applying n periods of U_F (dagger = false) or of U_F^dagger
// (dagger = true) in an order that respects every gate dependency of the
// brickwork.  Gate-table index: bond b for G_b, (L-1) + b for G_b^dagger.
// With with_slots, every op also names a reduction slot (local to the pass,
// pass.sbond maps it to the bond; used by the reverse pass of the gradient,
// which accumulates a bond's overlap matrix right before undoing that
// bond's gate).  The tile must hold at most FL_MAX_SLOTS bonds.  A pass has
// at most max_groups register groups (gates that do not fit wait for a later
// pass).
std::vector<fl_pass> plan_sweep(const fl_geom& g, int n, bool dagger, bool with_slots,
                                int max_gates_per_pass, PlanStats* st = nullptr, int max_groups = FL_MAX_GROUPS);

// Passes that visit every bond exactly once (one group per bond, op slot =
// global bond index, no gate); the first pass has flags = 1 (also reduce the
// norm).
std::vector<fl_pass> plan_cover(const fl_geom& g);

// The same cover with each pass's bonds packed into register groups of g.R
// consecutive tile bits: a group with first bit u0 holds the bonds on bits
// (u0 + i, u0 + i + 1), i = 0 .. R-2 (op bit i, op slot = bond, no gate).
std::vector<fl_pass> plan_cover_groups(const fl_geom& g);

// Flatten a plan into int32 words (for inspection and host-side tests):
// [C, W, R, npasses, {h, ngroups, flags, {u0, nops, {opi, opg, ops}*}*}*]
void serialize_plan(const fl_geom& g, const std::vector<fl_pass>& plan, std::vector<int>& out);

}  // namespace fl
