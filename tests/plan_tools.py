"""Host-side readers of the flattened plans returned by fl_plan_query (test helpers)."""
from __future__ import annotations


def parse_plan(words):
    words = [int(w) for w in words]
    C, W, R, npasses = words[:4]
    i = 4
    passes = []
    for _ in range(npasses):
        h, ng, flags = words[i:i + 3]
        i += 3
        groups = []
        for _ in range(ng):
            u0, nops = words[i:i + 2]
            i += 2
            ops = []
            for _ in range(nops):
                ops.append(tuple(words[i:i + 3]))
                i += 3
            groups.append((u0, ops))
        passes.append((h, flags, groups))
    assert i == len(words)
    return C, W, R, passes


def phys_bit(u, C, h):
    return u if u < C else h + (u - C)


def gate_sequence(L, words):
    """Execution order of a sweep plan as (bond, gate_index, slot) triples,
    checking that every op sits inside its tile and register group and acts
    on two chain-adjacent bits."""
    C, W, R, passes = parse_plan(words)
    K = C + W
    nb = L - 1
    seq = []
    for h, _, groups in passes:
        if W > 0:
            assert C <= h and h + W <= L
        for u0, ops in groups:
            assert 0 <= u0 and u0 + R <= K
            for i, g, slot in ops:
                assert 0 <= i <= R - 2
                u = u0 + i
                p, p1 = phys_bit(u, C, h), phys_bit(u + 1, C, h)
                assert p1 == p + 1, "gate bits not adjacent on the chain"
                b = L - 2 - p
                assert 0 <= b < nb
                assert g in (b, nb + b), "gate-table index does not match the bond"
                seq.append((b, g, slot))
    return seq


def check_trace_equivalent(L, bonds, n, dagger):
    """The gate word equals the brickwork U_F^n (or (U_F^dagger)^n) in the
    trace monoid of commuting gates: gates on non-adjacent bonds commute, so
    two words are the same circuit iff every bond occurs n times and, for
    every adjacent pair (b, b+1), the projection onto {b, b+1} is the same
    alternation as in the layer-by-layer circuit."""
    nb = L - 1
    for b in range(nb):
        assert bonds.count(b) == n, f"bond {b} applied {bonds.count(b)} times, want {n}"

    def first_layer(b):
        return (b % 2 == 0) if dagger else (b % 2 == 1)

    for b in range(nb - 1):
        proj = [x for x in bonds if x in (b, b + 1)]
        f, o = (b, b + 1) if first_layer(b) else (b + 1, b)
        assert proj == [f, o] * n, f"order of bonds {b},{b + 1} differs from the brickwork"
