"""CPU check of the link tables behind the FP64 staple loads.

The FP64 over-improved staples load each orientation's ten distinct links in a
fixed order, given by the tables take_mu / take_a / take_bu / take_bd of
csrc/vsm_kernels_impl.h (link k of the order is U_mu or U_nu at
x + a mu + b nu, b for +nu or -nu).  The paths they serve are the plaquette
and the three rectangles of Eq. (over-improvement) through x + mu, one
orientation of nu at a time.  This test reads the tables from the source and
checks that they name exactly the links of those paths, each once, in the
documented order, with the links shared by the updates of x and x + 2 mu
(same annealing subset) next to each other.  The GPU parity tests check the
arithmetic built on them."""
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_2203_09764_amd", "csrc", "vsm_kernels_impl.h")

# The ten distinct links of the four paths of the +nu orientation (the paths
# of the -nu orientation walk nu backwards), as (direction is mu, a, b) in
# x + a mu + b nu.  Letters as in the source comments.
PLUS = {
    "A": (False, 0, 0), "B": (True, 0, 1), "C": (False, 1, 0), "D": (False, 0, 1),
    "E": (True, 0, 2), "F": (False, 1, 1), "G": (True, 1, 1), "H": (False, 2, 0),
    "M": (False, -1, 0), "N": (True, -1, 1),
}
MINUS = {
    "A": (False, 0, -1), "B": (True, 0, -1), "C": (False, 1, -1), "D": (False, 0, -2),
    "E": (True, 0, -2), "F": (False, 1, -2), "G": (True, 1, -1), "H": (False, 2, -1),
    "M": (False, -1, -1), "N": (True, -1, -1),
}


def _paths(orient):
    """Every link the four paths of one orientation multiply, from the path
    definitions: steps of +-mu and +-nu from x to x + mu."""
    s = 1 if orient == "+" else -1
    steps = {
        "plaquette": [("n", s), ("m", 1), ("n", -s)],
        "1x2": [("n", s), ("n", s), ("m", 1), ("n", -s), ("n", -s)],
        "2x1 left": [("n", s), ("m", 1), ("m", 1), ("n", -s), ("m", -1)],
        "2x1 middle": [("m", -1), ("n", s), ("m", 1), ("m", 1), ("n", -s)],
    }
    links = set()
    for path in steps.values():
        a = b = 0
        for d, k in path:
            # a step +d uses the link at the current site, a step -d the link
            # at the site it arrives at
            if d == "m":
                links.add((True, a if k > 0 else a - 1, b))
                a += k
            else:
                links.add((False, a, b if k > 0 else b - 1))
                b += k
        assert (a, b) == (1, 0)
    return links


def _table(name, text):
    m = re.search(r"constexpr\s+\w+\s+" + name + r"\s*\(int k\)\s*\{\s*constexpr\s+(\w+)\s+t\[10\]\s*=\s*\{([^}]*)\}",
                  text)
    assert m, name
    vals = [v.strip() for v in m.group(2).split(",")]
    if m.group(1) == "bool":
        return [v == "true" for v in vals]
    return [int(v) for v in vals]


def _order():
    text = open(SRC).read()
    mu, a, bu, bd = (_table(n, text) for n in ("take_mu", "take_a", "take_bu", "take_bd"))
    plus = [(mu[k], a[k], bu[k]) for k in range(10)]
    minus = [(mu[k], a[k], bd[k]) for k in range(10)]
    return plus, minus


# K = U_mu(x+mu) and L = U_mu(x-mu), on the paths of every nu, are loaded once
# per update by the caller
K, L = (True, 1, 0), (True, -1, 0)


def test_letters_are_the_links_of_the_paths():
    assert set(PLUS.values()) | {K, L} == _paths("+")
    assert set(MINUS.values()) | {K, L} == _paths("-")
    assert K not in PLUS.values() and L not in MINUS.values()


def test_tables_load_every_link_once_in_the_documented_order():
    plus, minus = _order()
    letters = [next(k for k, v in PLUS.items() if v == t) for t in plus]
    assert sorted(letters) == sorted(PLUS)
    assert "".join(letters) == "DEFBAHNGMC"
    # the same letter at the same position in both orientations
    assert [MINUS[c] for c in letters] == minus


def test_links_shared_with_the_update_two_rows_on_are_adjacent():
    """x + 2 mu is in the same subset as x; its A, N, M are x's H, G, C."""
    def shifted(t):
        is_mu, a, b = t
        return (is_mu, a + 2, b)
    for table in (PLUS, MINUS):
        for x_letter, partner_letter in (("H", "A"), ("G", "N"), ("C", "M")):
            assert table[x_letter] == shifted(table[partner_letter])
    plus, _ = _order()
    letters = "".join(next(k for k, v in PLUS.items() if v == t) for t in plus)
    for pair in ("AH", "NG", "MC"):
        i = letters.index(pair[0])
        assert letters[i + 1] == pair[1]
