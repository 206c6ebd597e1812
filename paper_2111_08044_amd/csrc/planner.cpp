// Greedy fusion planner for the brickwork circuit (the gate fusion of Sec. II
// and the local-qubit remapping that the paper does with axis swaps, done here
// by choosing which high bits a tile spans).
//
// Dependencies.  Write a = 0 for bonds of the layer applied first in each
// period and a = 1 for the other layer (forward: first layer = odd b, Eq. (4);
// U_F^dagger: first layer = even b).  The k-th application of bond b sits in
// global layer 2k + a_b.  It may run once every neighbouring bond q = b +- 1
// (which touches one of its sites) has completed all of its applications in
// earlier layers, i.e. cnt[q] >= k + a_b, and no application of q in a later
// layer has run (guaranteed by q's own rule).  Ready bonds are never
// neighbours, so a whole round of ready bonds can be applied in any order.
//
// A pass picks the high window h whose tile bit set admits the most ready
// gates (repeating rounds inside the tile, which time-blocks several periods
// into one sweep), then packs the pass's gate list into register groups.
#include "planner.h"

#include <algorithm>
#include <cstring>

namespace fl {

fl_geom make_geom(int L, int kmax, int r, int lowbits) {
    fl_geom g;
    g.L = L;
    if (L <= kmax) {
        g.C = L;
        g.W = 0;
    } else {
        g.C = lowbits;
        g.W = kmax - lowbits;
    }
    g.K = g.C + g.W;
    g.R = std::min(r, g.K);
    return g;
}

namespace {

struct Gate {
    int bond;
    int u;     // tile-local bit (gate on u, u+1)
    int gidx;
    int slot;
};

struct Sched {
    int L, nb, n;
    std::vector<int> cnt, off;
    bool ready(int b) const {
        if (cnt[b] >= n) return false;
        const int need = cnt[b] + off[b];
        if (b > 0 && cnt[b - 1] < need) return false;
        if (b + 1 < nb && cnt[b + 1] < need) return false;
        return true;
    }
};

bool bond_in_tile(const fl_geom& g, int h, int b) {
    const int p = g.L - 2 - b;
    const int u = fl_local_bit(p, g.C, g.W, h);
    const int u1 = fl_local_bit(p + 1, g.C, g.W, h);
    return u >= 0 && u1 == u + 1;
}

// Apply rounds of ready gates inside tile window h; returns the bonds in order.
std::vector<int> run_tile(const fl_geom& g, int h, Sched& s, int cap) {
    std::vector<int> out;
    std::vector<int> round;
    while ((int)out.size() < cap) {
        round.clear();
        for (int b = 0; b < s.nb; ++b)
            if (bond_in_tile(g, h, b) && s.ready(b)) round.push_back(b);
        if (round.empty()) break;
        for (int b : round) {
            if ((int)out.size() >= cap) break;
            s.cnt[b]++;
            out.push_back(b);
        }
    }
    return out;
}

// Pack an ordered gate list into register groups.  A gate may join the
// current group only if no earlier gate left for later shares one of its
// bits (then it commutes with everything it overtakes).  Returns the gates
// that did not fit into max_groups groups.
std::vector<Gate> pack_groups(const fl_geom& g, std::vector<Gate> rem, fl_pass& pd, int max_groups) {
    pd.ngroups = 0;
    while (!rem.empty() && pd.ngroups < max_groups) {
        int best_u0 = -1;
        std::vector<int> best;
        for (int u0 = 0; u0 + g.R <= g.K; ++u0) {
            unsigned blocked = 0;
            std::vector<int> take;
            for (int i = 0; i < (int)rem.size(); ++i) {
                const unsigned m = 3u << rem[i].u;
                const bool fits = rem[i].u >= u0 && rem[i].u + 1 < u0 + g.R;
                if ((m & blocked) == 0 && fits && (int)take.size() < FL_MAX_OPS)
                    take.push_back(i);
                else
                    blocked |= m;
            }
            if ((int)take.size() > (int)best.size()) {
                best = take;
                best_u0 = u0;
            }
        }
        const int gi = pd.ngroups++;
        pd.u0[gi] = (int8_t)best_u0;
        pd.nops[gi] = (int8_t)best.size();
        std::vector<char> used(rem.size(), 0);
        for (int k = 0; k < (int)best.size(); ++k) {
            const Gate& q = rem[best[k]];
            pd.opi[gi][k] = (int8_t)(q.u - best_u0);
            pd.opg[gi][k] = (int16_t)q.gidx;
            pd.ops[gi][k] = (int16_t)q.slot;
            used[best[k]] = 1;
        }
        std::vector<Gate> next;
        for (int i = 0; i < (int)rem.size(); ++i)
            if (!used[i]) next.push_back(rem[i]);
        rem.swap(next);
    }
    return rem;
}

// The kernels apply a group's ops two at a time; an odd count costs a copy of
// the register group after the last op.  Shift ops across the boundary of
// consecutive groups, which keeps the pass's op sequence unchanged, wherever
// the op's bits lie inside the other group's register bits, so that fewer
// groups have odd counts; groups left empty are dropped (one LDS exchange
// less).
void balance_groups(const fl_geom& g, fl_pass& pd) {
    auto fits = [&](int gi, int u) { return u >= pd.u0[gi] && u + 1 < pd.u0[gi] + g.R; };
    auto set_op = [&](int gi, int k, int u, int16_t gate, int16_t slot) {
        pd.opi[gi][k] = (int8_t)(u - pd.u0[gi]);
        pd.opg[gi][k] = gate;
        pd.ops[gi][k] = slot;
    };
    for (int gi = 0; gi + 1 < pd.ngroups; ++gi) {
        if (!(pd.nops[gi] & 1)) continue;
        const int a = gi, b = gi + 1;
        const int kl = pd.nops[a] - 1;
        const int ul = pd.u0[a] + pd.opi[a][kl];
        if (fits(b, ul) && pd.nops[b] < FL_MAX_OPS) {
            // the last op of a becomes the first op of b
            for (int k = pd.nops[b]; k > 0; --k) {
                pd.opi[b][k] = pd.opi[b][k - 1];
                pd.opg[b][k] = pd.opg[b][k - 1];
                pd.ops[b][k] = pd.ops[b][k - 1];
            }
            set_op(b, 0, ul, pd.opg[a][kl], pd.ops[a][kl]);
            pd.nops[b]++;
            pd.nops[a]--;
            continue;
        }
        if (pd.nops[b] == 0) continue;
        const int uf = pd.u0[b] + pd.opi[b][0];
        if (fits(a, uf) && pd.nops[a] < FL_MAX_OPS) {
            // the first op of b becomes the last op of a
            set_op(a, pd.nops[a], uf, pd.opg[b][0], pd.ops[b][0]);
            pd.nops[a]++;
            for (int k = 0; k + 1 < pd.nops[b]; ++k) {
                pd.opi[b][k] = pd.opi[b][k + 1];
                pd.opg[b][k] = pd.opg[b][k + 1];
                pd.ops[b][k] = pd.ops[b][k + 1];
            }
            pd.nops[b]--;
        }
    }
    int out = 0;
    for (int gi = 0; gi < pd.ngroups; ++gi) {
        if (pd.nops[gi] == 0) continue;
        if (out != gi) {
            pd.u0[out] = pd.u0[gi];
            pd.nops[out] = pd.nops[gi];
            for (int k = 0; k < pd.nops[gi]; ++k) {
                pd.opi[out][k] = pd.opi[gi][k];
                pd.opg[out][k] = pd.opg[gi][k];
                pd.ops[out][k] = pd.ops[gi][k];
            }
        }
        ++out;
    }
    for (int gi = out; gi < pd.ngroups; ++gi) pd.nops[gi] = 0;
    pd.ngroups = out;
}

// Passes the plain greedy rule (the window admitting the most gates) needs to
// finish the circuit from state s.
int greedy_passes(const fl_geom& g, const std::vector<int>& windows, Sched s, int cap) {
    long long left = 0;
    for (int b = 0; b < s.nb; ++b) left += s.n - s.cnt[b];
    int passes = 0;
    while (left > 0) {
        int best = 0;
        Sched best_s;
        for (int h : windows) {
            Sched t = s;
            const int got = (int)run_tile(g, h, t, cap).size();
            if (got > best) {
                best = got;
                best_s = std::move(t);
            }
        }
        if (best == 0) return 1 << 20;   // cannot happen for a valid circuit
        s = std::move(best_s);
        left -= best;
        ++passes;
    }
    return passes;
}

}  // namespace

std::vector<fl_pass> plan_sweep(const fl_geom& g, int n, bool dagger, bool with_slots,
                                int max_gates_per_pass, PlanStats* st, int max_groups) {
    if (max_groups < 1 || max_groups > FL_MAX_GROUPS) max_groups = FL_MAX_GROUPS;
    std::vector<fl_pass> plan;
    const int L = g.L, nb = L - 1;
    Sched s;
    s.L = L;
    s.nb = nb;
    s.n = n;
    s.cnt.assign(nb, 0);
    s.off.resize(nb);
    for (int b = 0; b < nb; ++b) {
        const bool first = dagger ? (b % 2 == 0) : (b % 2 == 1);
        s.off[b] = first ? 0 : 1;
    }
    std::vector<int> windows;
    if (g.W == 0)
        windows.push_back(g.C);
    else
        for (int h = g.C; h + g.W <= L; ++h) windows.push_back(h);

    long long total = (long long)n * nb, done = 0;
    while (done < total) {
        // One-step lookahead: take the window after which the greedy rule
        // finishes in the fewest passes; ties go to the window that applies
        // more gates now, then to the lower window.
        int best_h = -1, best_cost = 1 << 30;
        std::vector<int> best;
        for (int h : windows) {
            Sched t = s;
            std::vector<int> got = run_tile(g, h, t, max_gates_per_pass);
            if (got.empty()) continue;
            const int cost = greedy_passes(g, windows, t, max_gates_per_pass);
            if (cost < best_cost || (cost == best_cost && got.size() > best.size())) {
                best_cost = cost;
                best = got;
                best_h = h;
            }
        }
        if (best.empty()) break;  // cannot happen for a valid circuit
        std::vector<Gate> gl;
        for (int b : best) {
            Gate q;
            q.bond = b;
            q.u = fl_local_bit(L - 2 - b, g.C, g.W, best_h);
            q.gidx = dagger ? nb + b : b;
            q.slot = with_slots ? b : -1;
            gl.push_back(q);
        }
        fl_pass pd;
        std::memset(&pd, 0, sizeof(pd));
        pd.h = best_h;
        std::vector<Gate> left = pack_groups(g, gl, pd, max_groups);
#if !defined(FL_NO_BALANCE)
        balance_groups(g, pd);
#endif
        if (with_slots) {
            // map the bonds of this pass to local reduction slots
            int map[64];
            for (int b = 0; b < 64; ++b) map[b] = -1;
            pd.nslots = 0;
            for (int gi = 0; gi < pd.ngroups; ++gi)
                for (int k = 0; k < pd.nops[gi]; ++k) {
                    const int b = pd.ops[gi][k];
                    if (map[b] < 0) {
                        map[b] = pd.nslots++;
                        pd.sbond[map[b]] = (int8_t)b;
                    }
                    pd.ops[gi][k] = (int16_t)map[b];
                }
        }
        // gates that did not fit are not applied in this pass
        for (int b : best) s.cnt[b]++;
        for (const Gate& q : left) s.cnt[q.bond]--;
        const long long applied = (long long)best.size() - (long long)left.size();
        done += applied;
        plan.push_back(pd);
        if (st) {
            st->passes++;
            st->gates += applied;
            st->groups += pd.ngroups;
        }
    }
    return plan;
}

std::vector<fl_pass> plan_cover(const fl_geom& g) {
    std::vector<fl_pass> plan;
    const int L = g.L, nb = L - 1;
    std::vector<char> covered(nb, 0);
    int left = nb;
    std::vector<int> windows;
    if (g.W == 0)
        windows.push_back(g.C);
    else
        for (int h = g.C; h + g.W <= L; ++h) windows.push_back(h);
    bool first = true;
    while (left > 0 || first) {
        int best_h = windows[0], best_n = -1;
        for (int h : windows) {
            int c = 0;
            for (int b = 0; b < nb; ++b)
                if (!covered[b] && bond_in_tile(g, h, b)) ++c;
            if (c > best_n) {
                best_n = c;
                best_h = h;
            }
        }
        fl_pass pd;
        std::memset(&pd, 0, sizeof(pd));
        pd.h = best_h;
        pd.flags = first ? 1 : 0;
        first = false;
        for (int b = 0; b < nb && pd.ngroups < FL_MAX_GROUPS; ++b) {
            if (covered[b] || !bond_in_tile(g, best_h, b)) continue;
            const int gi = pd.ngroups++;
            pd.u0[gi] = (int8_t)fl_local_bit(L - 2 - b, g.C, g.W, best_h);
            pd.nops[gi] = 1;
            pd.opi[gi][0] = 0;
            pd.opg[gi][0] = -1;
            pd.ops[gi][0] = (int16_t)b;
            covered[b] = 1;
            --left;
        }
        plan.push_back(pd);
    }
    return plan;
}

std::vector<fl_pass> plan_cover_groups(const fl_geom& g) {
    std::vector<fl_pass> plan = plan_cover(g);
    for (fl_pass& pd : plan) {
        // (tile bit, bond) of every bond of the pass, by tile bit
        std::vector<std::pair<int, int>> bonds;
        for (int gi = 0; gi < pd.ngroups; ++gi) bonds.emplace_back((int)pd.u0[gi], (int)pd.ops[gi][0]);
        std::sort(bonds.begin(), bonds.end());
        fl_pass q;
        std::memset(&q, 0, sizeof(q));
        q.h = pd.h;
        q.flags = pd.flags;
        size_t k = 0;
        while (k < bonds.size()) {
            const int u0 = std::min(bonds[k].first, g.K - g.R);
            const int gi = q.ngroups++;
            q.u0[gi] = (int8_t)u0;
            int n = 0;
            while (k < bonds.size() && bonds[k].first + 1 < u0 + g.R) {
                q.opi[gi][n] = (int8_t)(bonds[k].first - u0);
                q.opg[gi][n] = -1;
                q.ops[gi][n] = (int16_t)bonds[k].second;
                ++n;
                ++k;
            }
            q.nops[gi] = (int8_t)n;
        }
        pd = q;
    }
    return plan;
}

void serialize_plan(const fl_geom& g, const std::vector<fl_pass>& plan, std::vector<int>& out) {
    out.clear();
    out.push_back(g.C);
    out.push_back(g.W);
    out.push_back(g.R);
    out.push_back((int)plan.size());
    for (const fl_pass& p : plan) {
        out.push_back(p.h);
        out.push_back(p.ngroups);
        out.push_back(p.flags);
        for (int gi = 0; gi < p.ngroups; ++gi) {
            out.push_back(p.u0[gi]);
            out.push_back(p.nops[gi]);
            for (int k = 0; k < p.nops[gi]; ++k) {
                out.push_back(p.opi[gi][k]);
                out.push_back(p.opg[gi][k]);
                const int sl = p.ops[gi][k];
                // report reduction slots as bond indices
                out.push_back((p.nslots > 0 && sl >= 0) ? (int)p.sbond[sl] : sl);
            }
        }
    }
}

}  // namespace fl
