"""Integer arithmetic as gate netlists: adders and multipliers on encrypted
bits, in the gate set of the batched kernels (NAND, AND, OR, XOR, MUX, ...).

ArctyrEX's frontend synthesises such circuits from C (Section 3.2) with a
cost model in which a MUX counts twice a two-input gate; a levelled circuit
then costs about one bootstrap batch per level (Section 4.2), so on a GPU its
depth sets the latency and its gate count the throughput.  Two designs of
each operation are built here, both little-endian over wire lists:

* adders: ripple carry (depth ~ bits) and a Sklansky parallel-prefix adder
  (depth 2 + log2(bits));
* multipliers: the array multiplier (one ripple row per partial-product
  row, depth ~ 6 * bits) and a Dadda tree multiplier (two levels per
  reduction stage, ~log_1.5(bits) stages) followed by a Sklansky adder on
  the two remaining rows.

A full adder is p = x ^ y, sum = p ^ z, carry = MUX(p, z, x): when x and y
differ the carry is z, otherwise it is x.  A prefix node combines
(G_hi, P_hi) with (G_lo, P_lo) into (MUX(P_hi, G_lo, G_hi), P_hi & P_lo),
exact because a propagating block never generates (P_hi = 1 forces
G_hi = 0 when p = x ^ y and g = x & y).
"""
from .inputs import Netlist, array_multiplier, ripple_adder


class _Timed:
    """Gate builder that tracks each wire's ASAP level (inputs at 0)."""

    def __init__(self, nl):
        self.nl = nl
        self.t = {}

    def at(self, w):
        return self.t.get(w, 0)

    def gate(self, op, a=0, b=0, c=0):
        ins = (a, b, c) if op == "MUX" else (a, b)
        w = self.nl.gate(op, a, b, c)
        self.t[w] = 1 + max(self.at(x) for x in ins)
        return w


def _prefix_combine(tb, hi, lo, need_p):
    """(G, P) of the concatenation of block hi above block lo.  None stands
    for a constant 0 (no generate, or a column with no bits)."""
    g_hi, p_hi = hi
    g_lo, p_lo = lo
    if g_lo is None or p_hi is None:
        g = g_hi
    elif g_hi is None:
        g = tb.gate("AND", p_hi, g_lo)
    else:
        g = tb.gate("MUX", p_hi, g_lo, g_hi)
    p = None
    if need_p and p_hi is not None and p_lo is not None:
        p = tb.gate("AND", p_hi, p_lo)
    return g, p


def _sklansky_sum(tb, cols):
    """Add columns of at most two bits each (cols[k] = wires of weight k).
    Returns one sum bit per column; the carry out of the top column is
    dropped (callers size cols so that it is zero or use the top column)."""
    w = len(cols)
    G, P = [], []
    for bits in cols:
        if len(bits) == 2:
            G.append(tb.gate("AND", bits[0], bits[1]))
            P.append(tb.gate("XOR", bits[0], bits[1]))
        elif len(bits) == 1:
            G.append(None)
            P.append(bits[0])
        elif not bits:
            G.append(None)
            P.append(None)
        else:
            raise ValueError("column holds more than two bits")
    p0 = list(P)
    s = 0
    while (1 << s) < w:
        nG, nP = list(G), list(P)
        for k in range(w):
            if (k >> s) & 1:
                j = ((k >> s) << s) - 1
                nG[k], nP[k] = _prefix_combine(tb, (G[k], P[k]),
                                               (G[j], P[j]),
                                               need_p=(k >> (s + 1)) > 0)
        G, P = nG, nP
        s += 1
    out = []
    for k in range(w):
        c = G[k - 1] if k else None
        if p0[k] is None and c is None:
            out.append(tb.gate("CONST0"))
        elif c is None:
            out.append(p0[k])
        elif p0[k] is None:
            out.append(c)
        else:
            out.append(tb.gate("XOR", p0[k], c))
    return out, G[w - 1]


def sklansky_adder(nl, a, b):
    """Parallel-prefix adder of two equal-length bit lists.  Returns the sum
    bits and the carry out, like ripple_adder."""
    if len(a) != len(b):
        raise ValueError("operands differ in width")
    tb = _Timed(nl)
    s, c = _sklansky_sum(tb, [[x, y] for x, y in zip(a, b)])
    return s, c


def _full_adder(tb, x, y, z):
    p = tb.gate("XOR", x, y)
    return tb.gate("XOR", p, z), tb.gate("MUX", p, z, x)


def tree_multiplier(nl, a, b):
    """n x n Dadda multiplier: AND partial products; stages that bring every
    column down to the next height of 2, 3, 4, 6, 9, 13, ... (each target is
    the previous times 3/2, rounded down), counting the carries that enter a
    column in the same stage; full adders take the earliest-ready bits of a
    column, a half adder (XOR, AND) removes a last excess bit; sums stay in
    their column, carries move up one.  A Sklansky adder then adds the two
    remaining rows.  Every stage reads only bits of the previous one, so it
    adds two levels.  Returns 2n product bits."""
    n = len(a)
    if len(b) != n:
        raise ValueError("operands differ in width")
    tb = _Timed(nl)
    w = 2 * n
    cols = [[] for _ in range(w)]
    for i in range(n):
        for j in range(n):
            cols[i + j].append(tb.gate("AND", a[j], b[i]))
    heights = [2]
    while heights[-1] < max(len(c) for c in cols):
        heights.append(heights[-1] * 3 // 2)
    for target in reversed(heights[:-1]):
        nxt = [[] for _ in range(w)]
        for k in range(w):
            col = sorted(cols[k], key=tb.at)
            h = len(col) + len(nxt[k])
            while h > target:
                if h - target >= 2:
                    s, c = _full_adder(tb, col.pop(0), col.pop(0), col.pop(0))
                    h -= 2
                else:
                    x, y = col.pop(0), col.pop(0)
                    s, c = tb.gate("XOR", x, y), tb.gate("AND", x, y)
                    h -= 1
                nxt[k].append(s)
                if k + 1 < w:
                    nxt[k + 1].append(c)
            nxt[k] += col
        cols = nxt
    out, _ = _sklansky_sum(tb, cols)
    return out


ADDERS = {"ripple": ripple_adder, "prefix": sklansky_adder}
MULTIPLIERS = {"array": array_multiplier, "tree": tree_multiplier}


def adder(bits=32, style="prefix"):
    """(netlist, io): io['a'], io['b'] operand wires, io['sum'] the
    bits + 1 sum wires (carry out last)."""
    nl = Netlist()
    a, b = nl.inputs(bits), nl.inputs(bits)
    s, c = ADDERS[style](nl, a, b)
    return nl, dict(a=a, b=b, sum=list(s) + [c])


def multiplier(bits=32, style="tree"):
    """(netlist, io): io['a'], io['b'] operand wires, io['prod'] the
    2 * bits product wires."""
    nl = Netlist()
    a, b = nl.inputs(bits), nl.inputs(bits)
    return nl, dict(a=a, b=b, prod=list(MULTIPLIERS[style](nl, a, b)))
