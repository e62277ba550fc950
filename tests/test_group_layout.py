"""Host checks of the group kernels' layout tables (code generator): the LDS
areas of a system are disjoint, every packed term sequence decodes to the
signed rates of its unknown in the reference evaluation's order, and every
reaction position's operand code names the reaction's species."""
import pytest

from paper_1611_02274_amd import codegen as cg
from paper_1611_02274_amd import inputs as I

CASES = [(32, False), (53, False), (32, True), (53, True)]


def _layout(n_sp, thermal):
    net = I.standard_network(n_sp)
    lanes = 32 if thermal else cg.group_lanes(n_sp)
    return net, cg._group_layout(net, lanes, thermal=thermal)


def _expected_terms(net, k, pos_of, neg):
    """Species k's signed rates: reaction by reaction, each reactant slot
    holding k subtracts q_j, then each product slot holding k adds it."""
    out = []
    for j in range(net.n_rx):
        out += [pos_of[j] + neg for s in net.reac[j] if int(s) == k]
        out += [pos_of[j] for s in net.prod[j] if int(s) == k]
    return out


@pytest.mark.parametrize("n_sp,thermal", CASES)
def test_lds_areas_disjoint(n_sp, thermal):
    net, G = _layout(n_sp, thermal)
    n, R, L = G["n"], G["R"], G["L"]
    q0 = G["off_q"]
    areas = [("C", 0, n + (2 if thermal else 1)),          # C, the [M] place (and T)
             ("+q", q0, q0 + R * L),
             ("zero", q0 + R * L, q0 + R * L + 1),
             ("scratch", G["off_red"], G["off_red"] + G["nu"]),
             ("-q", q0 + G["neg"], q0 + G["neg"] + R * L)]
    if thermal:
        areas.append(("energy", G["off_e1"], G["off_e2"] + n))
        assert G["off_e1"] - G["off_red"] >= 11, "room for the RKC recurrence"
        assert G["off_e2"] >= G["off_e1"] + n
    spans = sorted((a, b, name) for name, a, b in areas if name != "energy")
    for (a0, b0, n0), (a1, b1, n1) in zip(spans, spans[1:]):
        assert b0 <= a1, f"{n0} overlaps {n1}"
    if thermal:   # the energy rows share the scratch, never the zero or the rates
        e0, e1 = G["off_e1"], G["off_e2"] + n
        assert e0 >= G["off_red"] and e1 <= q0 + G["neg"]
    assert spans[-1][1] <= G["lds_per_system"]
    for off in (G["off_q"], G["off_red"], G["lds_per_system"]) + (
            (G["off_e1"], G["off_e2"]) if thermal else ()):
        assert off % 2 == 0, "16-byte aligned (pairs are read as one)"


@pytest.mark.parametrize("n_sp,thermal", CASES)
def test_term_sequences_decode(n_sp, thermal):
    net, G = _layout(n_sp, thermal)
    L, bits, per_word, chunk = G["L"], G["bits"], G["per_word"], G["chunk"]
    sentinel, neg = G["sentinel"], G["neg"]
    pos_of = [-1] * net.n_rx
    for p, j in enumerate(G["rx_of"]):
        if j >= 0:
            assert pos_of[j] == -1
            pos_of[j] = p
    assert min(pos_of) >= 0, "every reaction has a position"
    owned = sorted(u for u in G["sp"] if u >= 0)
    assert owned == list(range(G["nu"])), "each unknown has exactly one slot"
    for r in range(L):
        codes = [(G["tc"][(t // per_word) * L + r] >> ((t % per_word) * bits)) & ((1 << bits) - 1)
                 for t in range(G["tot"])]
        cut = G["bnd"][r] * chunk
        for part, u in ((codes[:cut], G["sp"][r]), (codes[cut:], G["sp"][L + r])):
            while part and part[-1] == sentinel:
                part = part[:-1]
            k = u - 1 if thermal else u          # species of the unknown (T: none)
            want = _expected_terms(net, k, pos_of, neg) if k >= 0 else []
            assert part == want, f"lane {r} unknown {u}"
        assert all(c == sentinel or c < sentinel or neg <= c < neg + sentinel for c in codes)


@pytest.mark.parametrize("n_sp,thermal", CASES)
def test_operand_codes(n_sp, thermal):
    net, G = _layout(n_sp, thermal)
    n, L = net.n_sp, G["L"]
    for p, j in enumerate(G["rx_of"]):
        code = G["rx"][p]
        if j < 0:
            assert code == 0
            continue
        ops = [code & 0xff, (code >> 8) & 0xff, (code >> 16) & 0xff, code >> 24]
        want = [int(net.reac[j][0]), int(net.reac[j][1]), int(net.prod[j][0]), int(net.prod[j][1])]
        assert ops == [s if s >= 0 else n for s in want]
        if n in (ops[1], ops[3]):
            assert p // L >= G["m_first"], "a [M] operand only in the slots that select it"
