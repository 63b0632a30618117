"""Process generator for g g -> t tbar + n g (build time).

Enumerates the tree-level Feynman diagrams, expands each diagram's colour
factor onto the colour-flow basis, shares the off-shell sub-currents between
diagrams, and emits a straight-line per-helicity program (C++ templated on the
real type) that fills the colour-flow amplitudes J_sigma.  This is the
"code generator" role of the event generator the paper builds on (Sec. 3.1:
the generator emits process-specific amplitude routines, called as external
subroutines).

Diagrams.  Gluons are labelled 0..ng-1 (particles 0, 1, 4, 5, 6).  A diagram
is the top line (from the outgoing top to the outgoing antitop) with an
ordered sequence of pure-gluon trees attached, one per top-gluon vertex; each
tree is a leaf, a three-gluon vertex joining two trees, or a four-gluon vertex
joining three.  The four-gluon vertex carries three colour structures with
different Lorentz parts; the program evaluates them as three separate pieces of
the same diagram.  Diagram counts for ng = 2..5: 3, 16, 123, 1240.

Colour.  With f^{abc} T^c = -i [T^a, T^b] a three-gluon node contributes the
commutator of its two subtrees, a four-gluon piece the nested commutators
[1,[2,3]], [2,[1,3]], [3,[1,2]]; the top line multiplies the tree factors in
attachment order.  Collecting the constant phases of the Feynman rules
(i g kappa per top vertex, i per top propagator, -i/p^2 per gluon propagator,
g f^{abc} per three-gluon vertex, -i g^2 per four-gluon vertex) leaves every
diagram with the common factor i times a sign (-1)^(k-1) (-1)^(#3-gluon nodes)
for k top vertices; the common factor i is dropped (it cancels in |M|^2).

Couplings.  Programs that form their vertex momenta themselves apply the
couplings inside the chain (g per three-gluon vertex, g^2 per four-gluon
vertex, g kappa per top-gluon vertex).  Programs that read the momentum
combinations of their vertices from the event record (`vertex_kin`) run at unit
g -- every diagram carries g^ng, restored on |M|^2 -- and take kappa at each
top-vertex closure as kappa^b for its b top-gluon vertices; the record's vertex
and propagator momenta already include the propagator denominators.  Either
way, evaluating the program at a new parameter point is a full re-evaluation
of the amplitude.

Closures.  A top-vertex closure ubar_L Jslash v_R uses the vector current of
its (row, column) pair where that pair closes several trees of a group, and is
associated as ubar_L (Jslash v_R) where Jslash v_R also starts a column current
of the program; a root closure contracts the t tbar current with its vertex
term by term, so that its products with subtree currents are shared.
"""
from fractions import Fraction
from functools import lru_cache
from itertools import permutations

GLUON_PARTICLE = (0, 1, 4, 5, 6)


def bits(mask):
    return [i for i in range(8) if mask >> i & 1]


def lowbit(mask):
    return mask & -mask


def submasks(mask):
    s = mask
    while s:
        yield s
        s = (s - 1) & mask


class Tree:
    """A pure-gluon tree (off-shell gluon current)."""

    __slots__ = ("kind", "kids", "mask", "piece", "key")

    def __init__(self, kind, kids=(), mask=0, piece=None):
        self.kind = kind            # 'leaf', 'v3', 'v4'
        self.kids = tuple(kids)
        self.mask = mask
        self.piece = piece          # for v4: 'A', 'B', 'C'
        if kind == "leaf":
            self.key = f"g{bits(mask)[0]}"
        else:
            inner = ",".join(k.key for k in self.kids)
            self.key = f"{kind}{piece or ''}({inner})"

    def n_v3(self):
        return (self.kind == "v3") + sum(k.n_v3() for k in self.kids)

    def __repr__(self):
        return self.key


@lru_cache(maxsize=None)
def trees(mask, split_v4=True):
    """All trees over the gluon set `mask` (four-gluon pieces split if asked)."""
    if mask & (mask - 1) == 0:
        return (Tree("leaf", (), mask),)
    out = []
    low = lowbit(mask)
    for s1 in submasks(mask):
        if not s1 & low or s1 == mask:
            continue
        s2 = mask ^ s1
        for t1 in trees(s1, split_v4):
            for t2 in trees(s2, split_v4):
                out.append(Tree("v3", (t1, t2), mask))
    for s1 in submasks(mask):
        if not s1 & low or s1 == mask:
            continue
        rest = mask ^ s1
        low2 = lowbit(rest)
        for s2 in submasks(rest):
            if not s2 & low2 or s2 == rest:
                continue
            s3 = rest ^ s2
            for t1 in trees(s1, split_v4):
                for t2 in trees(s2, split_v4):
                    for t3 in trees(s3, split_v4):
                        if split_v4:
                            for piece in "ABC":
                                out.append(Tree("v4", (t1, t2, t3), mask, piece))
                        else:
                            out.append(Tree("v4", (t1, t2, t3), mask))
    return tuple(out)


def diagrams(ng, split_v4=True):
    """Ordered sequences of trees covering all gluons (top line attachments)."""
    full = (1 << ng) - 1
    out = []

    def rec(covered, seq):
        rest = full ^ covered
        for s in submasks(rest):
            for t in trees(s, split_v4):
                if s == rest:
                    out.append(seq + (t,))
                else:
                    rec(covered | s, seq + (t,))

    rec(0, ())
    return out


def n_diagrams(ng):
    return len(diagrams(ng, split_v4=False))


# ------------------------------------------------------------------- colour

def _comm(a, b):
    out = {}
    for wa, ca in a.items():
        for wb, cb in b.items():
            out[wa + wb] = out.get(wa + wb, 0) + ca * cb
            out[wb + wa] = out.get(wb + wa, 0) - ca * cb
    return {w: c for w, c in out.items() if c}


def _prod(a, b):
    out = {}
    for wa, ca in a.items():
        for wb, cb in b.items():
            out[wa + wb] = out.get(wa + wb, 0) + ca * cb
    return {w: c for w, c in out.items() if c}


def tree_colour(t):
    if t.kind == "leaf":
        return {(bits(t.mask)[0],): 1}
    c = [tree_colour(k) for k in t.kids]
    if t.kind == "v3":
        return _comm(c[0], c[1])
    if t.piece == "A":
        return _comm(c[0], _comm(c[1], c[2]))
    if t.piece == "B":
        return _comm(c[1], _comm(c[0], c[2]))
    return _comm(c[2], _comm(c[0], c[1]))


def diagram_colour(seq):
    """Coefficients of the diagram on the colour-flow basis, phases included
    (up to the common factor i)."""
    col = {(): 1}
    for t in seq:
        col = _prod(col, tree_colour(t))
    k = len(seq)
    sign = (-1) ** (k - 1) * (-1) ** sum(t.n_v3() for t in seq)
    return {w: sign * c for w, c in col.items()}


def flows(ng):
    return list(permutations(range(ng)))


# ---------------------------------------------------- colour matrix (own)

def colour_matrix_loops(ng, nc=3):
    """Colour matrix by index-loop counting (independent of any trace recursion).

    Each gluon propagator is T^a_{ij} T^a_{kl} = 1/2 (d_il d_kj - d_ij d_kl / N).
    For the product (T^s)_{ij} conj((T^r)_{ij}) summed over colours, choose for
    each gluon either the first (flow) or the second (U(1)) term; the Kronecker
    deltas then close into a number L of index loops, each worth N, and the
    term carries (1/2)^n (-1/N)^u for u U(1) choices."""
    words = flows(ng)
    n = ng
    # fundamental index slots: amplitude chain i=x0 -> x1 -> ... -> xn=j, and the
    # conjugate chain (reversed product) closing j back to i.
    cf = []
    for s in words:
        row = []
        for r in words:
            total = Fraction(0)
            for choice in range(1 << n):
                # nodes: ('a', pos) slots of amplitude matrices, ('c', pos) of conjugate
                parent = {}

                def find(x):
                    while parent.setdefault(x, x) != x:
                        parent[x] = parent[parent[x]]
                        x = parent[x]
                    return x

                def union(a, b):
                    ra, rb = find(a), find(b)
                    if ra != rb:
                        parent[ra] = rb

                # amplitude: (T^{s1})_{a0 a1'} (T^{s2})_{a1 a2'} ... row/col index per
                # matrix position p: row ('ar', p), col ('ac', p); chain: ac p == ar p+1
                for p in range(n - 1):
                    union(("ac", p), ("ar", p + 1))
                # conjugate of (T^r)_{ij}: conj(T^a)_{kl} = (T^a)_{lk}; the conjugate
                # chain with positions q: conj matrix q has row ('cr', q) col ('cc', q)
                for q in range(n - 1):
                    union(("cc", q), ("cr", q + 1))
                # open ends: i = ar 0 = cr 0, j = ac n-1 = cc n-1
                union(("ar", 0), ("cr", 0))
                union(("ac", n - 1), ("cc", n - 1))
                u = 0
                for g in range(n):
                    pa = s.index(g)
                    pc = r.index(g)
                    # amplitude factor (T^a)_{ar pa, ac pa}; conjugate factor is
                    # (T^a)_{cc pc, cr pc} (transposed by the conjugation)
                    if choice >> g & 1:     # -1/N d_{row col} d_{row' col'}
                        u += 1
                        union(("ar", pa), ("ac", pa))
                        union(("cc", pc), ("cr", pc))
                    else:                   # d_{ar, cr'} d_{cc', ac}
                        union(("ar", pa), ("cr", pc))
                        union(("cc", pc), ("ac", pa))
                nodes = [("ar", p) for p in range(n)] + [("ac", p) for p in range(n)] + \
                        [("cr", p) for p in range(n)] + [("cc", p) for p in range(n)]
                loops = len({find(x) for x in nodes})
                total += Fraction(1, 2 ** n) * Fraction(-1, nc) ** u * Fraction(nc) ** loops
            row.append(total)
        cf.append(row)
    return cf


# -------------------------------------------------------------- emission

def popcount(m):
    return bin(m).count("1")


def closing(seq):
    """Where a diagram's amplitude is closed.

    ('leaf', j): all blocks are single gluons; closed at top vertex j.
    ('ttg', U, j): closed at the top-gluon vertex of block j, the first of the
                   largest gluon trees (over the gluon set U).
    ('root', U, None): a single tree spans every gluon; closed at that tree's
                   root gluon vertex against the t tbar current; U is the set
                   of the root's largest child."""
    sizes = [popcount(t.mask) for t in seq]
    big = max(sizes)
    if big == 1:
        return ("leaf", None, (len(seq) - 1) // 2)
    j = sizes.index(big)
    if len(seq) == 1:
        kids = seq[0].kids
        ks = [popcount(k.mask) for k in kids]
        return ("root", kids[ks.index(max(ks))].mask, None)
    return ("ttg", seq[j].mask, j)


class Emitter:
    """Straight-line per-helicity program, grouped by closing tree.

    Every diagram is closed at one vertex (see `closing`): the amplitude is
    the contraction at that vertex of the row current from the top
    (L = ubar Gamma S Gamma S ...), the column current from the antitop
    (R = ... S Gamma S Gamma v) and the gluon tree attached there, or, for a
    tree spanning all gluons, of the tree's root children with the t tbar
    current.  Diagrams are grouped by the gluon set of their closing tree, and
    the sub-currents a group builds are private to it (rebuilt if another group
    needs them), so every intermediate dies at the end of its group; the
    external wavefunctions, the t tbar current and the single-gluon row and
    column currents are shared by all groups."""

    def __init__(self, ng, global_leaf_lr=True, kpoly=False, flow_range=None, merge_flows=True,
                 vertex_kin=False):
        self.ng = ng
        # vertex_kin: three-gluon vertices and top-line propagators read their
        # momentum combinations from the event record (V, QL, QR) instead of
        # forming them from the gluon-set momenta P in the program
        self.vertex_kin = vertex_kin
        # amplitudes of a closing group with the same (flow, sign) pattern over
        # several flows are summed first and the sum added to those flows once
        self.merge_flows = merge_flows
        self.pending = {}
        self.kpoly = kpoly          # accumulate J per power of kappa (J[(k-1)*K + w])
        # (lo, hi): accumulate only the flows lo <= w < hi, into J[w - lo]; diagrams
        # with no term there are left out, and so are the currents only they use
        self.flow_range = flow_range
        self.full = (1 << ng) - 1
        self.lines = []
        self.nvar = 0
        self.P_needed = set()      # incoming momentum sums entering the program (without vertex_kin)
        self.V_needed = set()      # (S1, S2) of three-gluon vertices: P1 - P2, P1 + 2 P2, P2 + 2 P1
        self.QL_needed = set()     # light-cone top-side propagator momenta (with vertex_kin)
        self.QR_needed = set()
        self.iP_needed = set()     # 1/P^2 of internal gluon lines
        self.qL_needed = set()     # top-side propagators: q = p_t - P(S), and 1/(q^2 - m^2)
        self.qR_needed = set()     # antitop-side propagators: q = P(S) - p_tbar, and 1/(q^2 - m^2)
        self.flows = flows(ng)
        self.flow_index = {w: i for i, w in enumerate(self.flows)}
        self.n_amp = 0
        self.n_jterms = 0
        self.counts = {"vvv": 0, "vvvv": 0, "ffv_row": 0, "ffv_col": 0, "ffv_amp": 0, "vector_current": 0,
                       "vvv_amp": 0, "vvvv_amp": 0, "tt_current": 0}
        self.lr_uses, self.vcur = {}, {}
        self.col_keys = set()   # column currents the program forms (see close_ttg)
        self.global_cache = {}
        self.cache = {}
        self.global_leaf_lr = global_leaf_lr

    def var(self, prefix):
        self.nvar += 1
        return f"{prefix}{self.nvar}"

    def emit(self, line):
        self.lines.append(line)

    def lookup(self, key):
        if key in self.cache:
            return self.cache[key]
        return self.global_cache.get(key)

    def vmom(self, t):
        """Momentum argument of the three-gluon vertex joining t's two subtrees."""
        m1, m2 = t.kids[0].mask, t.kids[1].mask
        if self.vertex_kin:
            self.V_needed.add((m1, m2))
            return f"k.V{m1}_{m2}"
        self.P_needed |= {m1, m2}
        return f"vvv_mom_of(k.P{m1}, k.P{m2})"

    # ---- gluon trees
    def tree(self, t):
        key = "T:" + t.key
        v = self.lookup(key)
        if v:
            return v
        if t.kind == "leaf":
            name = f"w.e{bits(t.mask)[0]}"
            self.global_cache[key] = name
            return name
        kids = [self.tree(k) for k in t.kids]
        self.iP_needed.add(t.mask)
        if t.kind == "v3":
            name = self.var("c")
            if self.vertex_kin:   # the record's vertex momenta carry 1/P^2; unit coupling
                self.emit(f"const v4<T> {name} = vvv({kids[0]}, {kids[1]}, {self.vmom(t)});")
            else:
                self.emit(f"const v4<T> {name} = vvv({kids[0]}, {kids[1]}, {self.vmom(t)}, c.g * k.iP{t.mask});")
            self.counts["vvv"] += 1
            self.cache[key] = name
            return name
        q = self.var("c")
        g2 = "" if self.vertex_kin else "c.g2 * "
        self.emit(f"const auto {q} = vvvv({kids[0]}, {kids[1]}, {kids[2]}, {g2}k.iP{t.mask});")
        self.counts["vvvv"] += 1
        inner = ",".join(k.key for k in t.kids)
        for p in "ABC":
            self.cache[f"T:v4{p}({inner})"] = f"{q}.{p}"
        return self.cache[key]

    # ---- top line currents
    def L(self, seq):
        """Row current ubar Gamma(T1) S Gamma(T2) S ... Gamma(Tj) S."""
        if not seq:
            return "w.ub"
        key = "L:" + "|".join(t.key for t in seq)
        v = self.lookup(key)
        if v:
            return v
        prev = self.L(seq[:-1])
        cur = self.tree(seq[-1])
        mask = 0
        for t in seq:
            mask |= t.mask
        self.qL_needed.add(mask)
        name = self.var("l")
        if self.vertex_kin:   # momentum and mass carry 1/(q^2 - m^2); unit coupling
            self.QL_needed.add(mask)
            self.emit(f"const sp<T> {name} = ffv_row({prev}, {cur}, k.QL{mask}, k.mQL{mask});")
        else:
            self.P_needed.add(mask)
            self.emit(f"const sp<T> {name} = ffv_row({prev}, {cur}, k.pt - k.P{mask}, k.mt, c.gk * k.iqL{mask});")
        self.counts["ffv_row"] += 1
        glob = self.global_leaf_lr and len(seq) == 1 and seq[0].kind == "leaf"
        (self.global_cache if glob else self.cache)[key] = name
        return name

    def R(self, seq):
        """Column current S Gamma(T1) S Gamma(T2) ... Gamma(Tk) v."""
        if not seq:
            return "w.v"
        key = "R:" + "|".join(t.key for t in seq)
        v = self.lookup(key)
        if v:
            return v
        nxt = self.R(seq[1:])
        cur = self.tree(seq[0])
        mask = 0
        for t in seq:
            mask |= t.mask
        self.qR_needed.add(mask)
        name = self.var("r")
        if self.vertex_kin:
            self.QR_needed.add(mask)
            self.emit(f"const sp<T> {name} = ffv_col({cur}, {nxt}, k.QR{mask}, k.mQR{mask});")
        else:
            self.P_needed.add(mask)
            self.emit(f"const sp<T> {name} = ffv_col({cur}, {nxt}, k.P{mask} - k.ptb, k.mt, c.gk * k.iqR{mask});")
        self.counts["ffv_col"] += 1
        glob = self.global_leaf_lr and len(seq) == 1 and seq[0].kind == "leaf"
        (self.global_cache if glob else self.cache)[key] = name
        return name

    def tt_current(self):
        v = self.global_cache.get("Jtt")
        if v:
            return v
        self.iP_needed.add(self.full)
        self.emit(f"const v4<T> jtt = tt_current(w.ub, w.v, c.gk * k.iP{self.full});")
        self.counts["tt_current"] += 1
        self.global_cache["Jtt"] = "jtt"
        return "jtt"

    # ---- amplitudes
    def wanted(self, seq):
        if self.flow_range is None:
            return True
        lo, hi = self.flow_range
        return any(lo <= self.flow_index[w] < hi for w in diagram_colour(seq))

    def accumulate(self, amp, seq):
        col = diagram_colour(seq)
        terms = []
        for w, c in sorted(col.items(), key=lambda x: self.flow_index[x[0]]):
            assert c in (1, -1), (seq, w, c)
            j = self.flow_index[w]
            if self.flow_range is not None:
                if not self.flow_range[0] <= j < self.flow_range[1]:
                    continue
                j -= self.flow_range[0]
            if self.kpoly:   # one top-gluon vertex per attached tree: kappa^len(seq)
                j += (len(seq) - 1) * len(self.flows)
            terms.append((j, c))
        if self.merge_flows and len(terms) > 1:
            # running sum per pattern, normalised so that its first flow enters with +
            s0 = terms[0][1]
            key = tuple((j, c * s0) for j, c in terms)
            name = self.pending.get(key)
            if name is None:
                name = self.var("s")
                self.pending[key] = name
                self.emit(f"cx<T> {name} = {'' if s0 > 0 else '-'}{amp};")
            else:
                self.emit(f"{name} = {name} {'+' if s0 > 0 else '-'} {amp};")
            return
        for j, c in terms:
            op = "+" if c > 0 else "-"
            self.emit(f"J[{j}] = J[{j}] {op} {amp};")
            self.n_jterms += 1

    def flush(self):
        """Add the group's pattern sums to their flows."""
        for key, name in self.pending.items():
            for j, c in key:
                self.emit(f"J[{j}] = J[{j}] {'+' if c > 0 else '-'} {name};")
                self.n_jterms += 1
        self.pending = {}

    def close_ttg(self, seq, j):
        if not self.wanted(seq):
            return
        left, right = self.L(seq[:j]), self.R(seq[j + 1:])
        cur = self.tree(seq[j])
        a = self.var("a")
        # with unit couplings in the currents the closure carries the top line's
        # kappa^(number of top-gluon vertices)
        gk = f"c.gkp[{len(seq)}]" if self.vertex_kin else "c.gk"
        pair = self.lr_key(seq, j)
        if self.lr_uses.get(pair, 0) >= 2:
            # the pair closes several gluon trees in this group: its vector
            # current ubar_L gamma^mu v_R is formed once, each closure is a dot
            v = self.vcur.get(pair)
            if v is None:
                v = self.var("v")
                self.emit(f"const v4<T> {v} = vector_current({left}, {right});")
                self.counts["vector_current"] += 1
                self.vcur[pair] = v
            self.emit(f"const cx<T> {a} = dot({cur}, {v}) * {gk};")
        elif "|".join(t.key for t in seq[j:]) in self.col_keys:
            # the column current through this vertex exists elsewhere in the
            # program: share its slashed product
            self.emit(f"const cx<T> {a} = ffv_amp_col({left}, {cur}, {right}, {gk});")
        else:
            self.emit(f"const cx<T> {a} = ffv_amp({left}, {cur}, {right}, {gk});")
        self.counts["ffv_amp"] += 1
        self.n_amp += 1
        self.accumulate(a, seq)

    @staticmethod
    def lr_key(seq, j):
        return (tuple(t.key for t in seq[:j]), tuple(t.key for t in seq[j + 1:]))

    def count_pairs(self, items):
        """Uses of each (row current, column current) pair by the top-vertex
        closures of one group."""
        self.lr_uses, self.vcur = {}, {}
        for seq, j in items:
            if self.wanted(seq):
                k = self.lr_key(seq, j)
                self.lr_uses[k] = self.lr_uses.get(k, 0) + 1

    def close_root(self, seq):
        if not self.wanted(seq):
            return
        t = seq[0]
        jtt = self.tt_current()
        kids = [self.tree(k) for k in t.kids]
        unit = self.vertex_kin or self.kpoly   # the vertex carries no coupling
        if t.kind == "v3":
            a = self.var("a")
            if unit:   # contracted term by term
                self.emit(f"const cx<T> {a} = vvv_close({jtt}, {kids[0]}, {kids[1]}, {self.vmom(t)});")
            else:
                self.emit(f"const cx<T> {a} = dot({jtt}, vvv({kids[0]}, {kids[1]}, {self.vmom(t)}, c.g));")
            self.counts["vvv_amp"] += 1
            self.n_amp += 1
            self.accumulate(a, seq)
            return
        inner = ",".join(k.key for k in t.kids)
        rkey = f"ROOT4:{inner}"
        q = self.cache.get(rkey)
        if q is None:
            q = self.var("c")
            if unit:
                self.emit(f"const auto {q} = vvvv_close({jtt}, {kids[0]}, {kids[1]}, {kids[2]});")
            else:
                self.emit(f"const auto {q} = vvvv({kids[0]}, {kids[1]}, {kids[2]}, c.g2);")
            self.counts["vvvv_amp"] += 1
            self.cache[rkey] = q
        a = self.var("a")
        if unit:
            self.emit(f"const cx<T> {a} = {q}.{t.piece};")
        else:
            self.emit(f"const cx<T> {a} = dot({jtt}, {q}.{t.piece});")
        self.n_amp += 1
        self.accumulate(a, seq)

    def group_keys(self):
        """Closing groups in program order: 'leaf', then gluon-set masks."""
        keys = set()
        for seq in diagrams(self.ng):
            kind, U, j = closing(seq)
            keys.add("leaf" if kind == "leaf" else U)
        return ["leaf"] * ("leaf" in keys) + sorted((k for k in keys if k != "leaf"), key=lambda m: (popcount(m), m))

    def column_keys(self, only=None):
        """Keys of the column currents a program over `only` forms."""
        e = Emitter(self.ng, self.global_leaf_lr, self.kpoly, self.flow_range, self.merge_flows, self.vertex_kin)
        e.col_keys = {None}   # no look-ahead of its own
        keys = set()
        plain_R = e.R

        def R(seq):
            if seq:
                keys.add("|".join(t.key for t in seq))
            return plain_R(seq)
        e.R = R
        e.program(only)
        return keys

    def program(self, only=None):
        """Emit the program; `only` restricts it to a set of group keys."""
        if (self.vertex_kin or self.kpoly) and not self.col_keys:
            self.col_keys = self.column_keys(only) or {None}
        diags = diagrams(self.ng)
        groups = {}
        leaf = []
        for seq in diags:
            kind, U, j = closing(seq)
            if kind == "leaf":
                leaf.append((seq, j))
            else:
                groups.setdefault(U, []).append((kind, seq, j))
        # single-gluon row/column currents and the t tbar current are shared
        # leaf-only diagrams: iterate over the column side first
        leaf.sort(key=lambda x: ([t.key for t in x[0][x[1] + 1:]], [t.key for t in x[0]]))
        if only is None or "leaf" in only:
            self.emit("// leaf-only diagrams")
            self.count_pairs(leaf)
            for seq, j in leaf:
                self.close_ttg(seq, j)
            self.flush()
        self.cache = {}
        for U in sorted(groups, key=lambda m: (popcount(m), m)):
            if only is not None and U not in only:
                continue
            items = groups[U]
            order = {t.key: i for i, t in enumerate(trees(U))}

            def anchor(it):
                kind, seq, j = it
                if kind == "ttg":
                    return order[seq[j].key]
                kids = seq[0].kids
                ks = [popcount(k.mask) for k in kids]
                return order[kids[ks.index(max(ks))].key]

            items.sort(key=lambda it: (anchor(it), it[0], [t.key for t in it[1]]))
            self.emit("MGRW_SCHED_BARRIER();")
            self.emit(f"// closing trees over gluons {bits(U)}")
            self.count_pairs([(seq, j) for kind, seq, j in items if kind == "ttg"])
            for kind, seq, j in items:
                if kind == "ttg":
                    self.close_ttg(seq, j)
                else:
                    self.close_root(seq)
            self.flush()
            self.cache = {}
        return self.lines


def split_groups(ng, chunks):
    """Consecutive closing groups partitioned into `chunks` parts of similar
    program size; each part is emitted as its own function (and kernel)."""
    keys = Emitter(ng).group_keys()
    sizes = [len(Emitter(ng).program({k})) for k in keys]
    total, parts, cur, acc = sum(sizes), [], [], 0
    for k, sz in zip(keys, sizes):
        cur.append(k)
        acc += sz
        if acc >= total * (len(parts) + 1) / chunks and len(parts) < chunks - 1:
            parts.append(cur)
            cur = []
    parts.append(cur)
    return [p for p in parts if p]


def bf16_bits(x):
    """bfloat16 bit pattern of x (round to nearest even), from its float32 bits."""
    import struct
    u = struct.unpack("<I", struct.pack("<f", x))[0]
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return u & 0xFFFF


def bf16_value(b):
    import struct
    return struct.unpack("<f", struct.pack("<I", b << 16))[0]


def bf16_split_table(num, kp):
    """Integer matrix num (K x K) padded with zeros to kp x kp, as two
    bfloat16 matrices hi + lo that sum to it exactly (row-major bit patterns)."""
    K = len(num)
    hi, lo = [], []
    for r in range(kp):
        for c in range(kp):
            v = num[r][c] if r < K and c < K else 0
            h = bf16_bits(float(v))
            rest = v - bf16_value(h)
            l = bf16_bits(float(rest))
            assert bf16_value(h) + bf16_value(l) == v, (v, h, l)
            hi.append(h)
            lo.append(l)
    return hi, lo


def emit_process(name, ng, chunks=1, fp64_split=None, vertex_kin=False):
    """C++ source of the process struct for g g -> t tbar + (ng-2) g.

    With chunks > 1 the per-helicity program is split into that many
    functions amplitude_part<C> over consecutive closing groups, each adding
    its diagrams to J; amplitude() zeroes J and runs all parts.

    fp64_split = (nch, nfr) also emits the program cut into nch chunks of
    closing groups times nfr equal ranges of colour flows,
    amplitude_fr<C, R>: chunk C's diagrams that have a term in flow range R,
    accumulated into that range only (J[w - R K/nfr]).  A diagram with terms in
    several ranges, and the currents it needs, appear in each of them; in
    exchange only K/nfr flow amplitudes are live at a time, which is what
    lets the program run in double precision.

    vertex_kin: the programs (not the kappa-polynomial one) read the momentum
    combinations of their vertices from the event record."""
    from math import factorial, gcd
    em = Emitter(ng, vertex_kin=vertex_kin)
    if chunks > 1:
        parts = split_groups(ng, chunks)
        part_ems = []
        for p in parts:
            e = Emitter(ng, vertex_kin=vertex_kin)
            e.program(set(p))
            part_ems.append(e)
        for e in part_ems:
            em.P_needed |= e.P_needed
            em.V_needed |= e.V_needed
            em.QL_needed |= e.QL_needed
            em.QR_needed |= e.QR_needed
            em.iP_needed |= e.iP_needed
            em.qL_needed |= e.qL_needed
            em.qR_needed |= e.qR_needed
            em.n_amp += e.n_amp
            em.n_jterms += e.n_jterms
            for kk, v in e.counts.items():
                em.counts[kk] += v
        body = None
    else:
        body = em.program()
    fr_ems = {}
    if fp64_split is not None:
        nch64, nfr = fp64_split
        kf = len(em.flows)
        assert kf % nfr == 0
        kr = kf // nfr
        parts64 = split_groups(ng, nch64)
        for c, p in enumerate(parts64):
            for r in range(nfr):
                e = Emitter(ng, flow_range=(r * kr, (r + 1) * kr), vertex_kin=vertex_kin)
                e.program(set(p))
                fr_ems[(c, r)] = (e, p)
                # every kinematic quantity the split program needs is in kin<T>
                assert e.V_needed <= em.V_needed and e.iP_needed <= em.iP_needed
                assert e.P_needed <= em.P_needed
                assert e.QL_needed <= em.QL_needed and e.QR_needed <= em.QR_needed
                assert e.qL_needed <= em.qL_needed and e.qR_needed <= em.qR_needed
    ek = None
    if chunks == 1:
        # kappa-polynomial form of the same diagrams (momenta from P in the program)
        ek = Emitter(ng, kpoly=True)
        kbody = ek.program()
        assert ek.iP_needed <= em.iP_needed
        assert ek.qL_needed <= em.qL_needed and ek.qR_needed <= em.qR_needed
        em.P_needed |= ek.P_needed
    K = len(em.flows)
    next_ = ng + 2
    cf = colour_matrix_loops(ng)
    den = 1
    for row in cf:
        for x in row:
            den = den * x.denominator // gcd(den, x.denominator)
    num = [[int(x * den) for x in row] for row in cf]

    P_masks = sorted(em.P_needed)
    V_pairs = sorted(em.V_needed)
    QL_masks = sorted(em.QL_needed)
    QR_masks = sorted(em.QR_needed)
    iP_masks = sorted(em.iP_needed)
    qL_masks = sorted(em.qL_needed)
    qR_masks = sorted(em.qR_needed)

    out = []
    w = out.append
    w(f"// Generated by paper_2312_07440_amd/gen/process.py -- g g -> t tbar + {ng - 2} g.")
    w(f"// {n_diagrams(ng)} Feynman diagrams, {K} colour flows, {1 << next_} helicity configurations.")
    w("// Per helicity: " + ", ".join(f"{v} {k}" for k, v in em.counts.items()) +
      f", {em.n_amp} amplitudes, {em.n_jterms} colour-flow accumulations.")
    w("#pragma once")
    w('#include "../mgrw_lorentz.h"')
    w("namespace mgrw {")
    w(f"struct {name} {{")
    w(f"  static constexpr int NG = {ng};")
    w(f"  static constexpr int NEXT = {next_};")
    w(f"  static constexpr int K = {K};")
    w(f"  static constexpr int NHEL = {1 << next_};")
    w(f"  static constexpr int NDIAG = {n_diagrams(ng)};")
    w(f"  static constexpr int CF_DEN = {den};")
    w(f"  static constexpr double NORM = 1.0 / (4.0 * 64.0 * {factorial(ng - 2)}.0 * {den}.0);")
    w("  // Helicity-independent kinematics of one event, formed in double precision")
    w("  // and rounded once: incoming momentum sums P of gluon sets and the top and")
    w("  // antitop momenta (for programs that form their vertex momenta), the")
    w("  // momentum combinations of three-gluon vertices (V<S1>_<S2>) and the top-line")
    w("  // propagator momenta in light-cone form (QL, QR) for programs that read them,")
    w("  // and the inverse propagator denominators.")
    w("  template <typename T> struct kin {")
    w("    T mt;")
    if P_masks:
        w("    r4<T> pt, ptb;")
    for m in P_masks:
        w(f"    r4<T> P{m};")
    for m1, m2 in V_pairs:
        w(f"    vvv_mom<T> V{m1}_{m2};")
    for m in QL_masks:
        w(f"    lc4<T> QL{m};")
        w(f"    T mQL{m};")
    for m in QR_masks:
        w(f"    lc4<T> QR{m};")
        w(f"    T mQR{m};")
    for m in iP_masks:
        w(f"    T iP{m};")
    for m in qL_masks:
        w(f"    T iqL{m};")
    for m in qR_masks:
        w(f"    T iqR{m};")
    w("  };")
    w("  template <typename T> struct basis {")
    for i in range(ng):
        w(f"    gluon_basis<T> g{i};")
    w("    fermion_basis<T> t, tb;")
    w("  };")
    w("  template <typename T> struct ext {")
    for i in range(ng):
        w(f"    pol4<T> e{i};")
    w("    sp<T> ub, v;")
    w("  };")
    w("  template <typename T, typename P>")
    w("  static MGRW_HD void kinematics(const P& p, double mt, kin<T>& k) {")
    w("    k.mt = T(mt);")
    if P_masks:
        w("    k.pt = {T(p[2][0]), T(p[2][1]), T(p[2][2]), T(p[2][3])};")
        w("    k.ptb = {T(p[3][0]), T(p[3][1]), T(p[3][2]), T(p[3][3])};")
    w("    double kin_in[NG][4];")
    for i, ip in enumerate(GLUON_PARTICLE[:ng]):
        sgn = "" if ip < 2 else "-"
        w(f"    for (int m = 0; m < 4; ++m) kin_in[{i}][m] = {sgn}p[{ip}][m];")
    allm = sorted(set(P_masks) | {m for pr in V_pairs for m in pr} | set(iP_masks) | set(qL_masks) | set(qR_masks))
    for m in allm:
        terms = " + ".join(f"kin_in[{i}][m]" for i in bits(m))
        w(f"    double S{m}[4]; for (int m = 0; m < 4; ++m) S{m}[m] = {terms};")
    for m in P_masks:
        w(f"    k.P{m} = {{T(S{m}[0]), T(S{m}[1]), T(S{m}[2]), T(S{m}[3])}};")
    full = (1 << ng) - 1
    for m1, m2 in V_pairs:
        # an internal vertex's combinations carry the propagator 1/P^2 of the
        # line they feed; the root vertex's (P1 + P2 = the t tbar line) do not
        u = m1 | m2
        f = "1.0" if u == full else (f"1.0 / (((S{u}[0] * S{u}[0] - S{u}[1] * S{u}[1]) - S{u}[2] * S{u}[2]) - "
                                     f"S{u}[3] * S{u}[3])")
        w(f"    {{ const double f = {f}; double d[4], b[4], c[4];")
        w(f"      for (int m = 0; m < 4; ++m) {{ d[m] = f * (S{m1}[m] - S{m2}[m]); "
          f"b[m] = f * (S{m1}[m] + 2.0 * S{m2}[m]); c[m] = f * (S{m2}[m] + 2.0 * S{m1}[m]); }}")
        w(f"      k.V{m1}_{m2} = {{{{T(d[0]), T(d[1]), T(d[2]), T(d[3])}}, {{T(b[0]), T(b[1]), T(b[2]), T(b[3])}}, "
          f"{{T(c[0]), T(c[1]), T(c[2]), T(c[3])}}}}; }}")
    for m in iP_masks:
        w(f"    k.iP{m} = T(1.0 / (((S{m}[0] * S{m}[0] - S{m}[1] * S{m}[1]) - S{m}[2] * S{m}[2]) - "
          f"S{m}[3] * S{m}[3]));")
    for side, m_list, qexpr in (("L", qL_masks, "p[2][m] - S{m}[m]"), ("R", qR_masks, "S{m}[m] - p[3][m]")):
        for m in m_list:
            w(f"    {{ double q[4]; for (int m = 0; m < 4; ++m) q[m] = {qexpr.format(m=m)};")
            w(f"      const double iq = 1.0 / ((((q[0] - q[3]) * (q[0] + q[3]) - q[1] * q[1]) - q[2] * q[2]) - mt * mt);")
            if m in (QL_masks if side == "L" else QR_masks):
                # momentum and mass of the numerator qslash + m, times the denominator
                w(f"      k.Q{side}{m} = {{T(iq * (q[0] + q[3])), T(iq * (q[0] - q[3])), T(iq * q[1]), T(iq * q[2])}};")
                w(f"      k.mQ{side}{m} = T(iq * mt);")
            w(f"      k.iq{side}{m} = T(iq); }}")
    w("  }")
    w("  template <typename T, typename P>")
    w("  static MGRW_HD void external_basis(const P& p, double mt, basis<T>& b) {")
    for i, ip in enumerate(GLUON_PARTICLE[:ng]):
        w(f"    b.g{i} = make_gluon_basis<T>(p[{ip}]);")
    w("    b.t = make_fermion_basis<T>(p[2], mt);")
    w("    b.tb = make_fermion_basis<T>(p[3], mt);")
    w("  }")
    w("  template <typename T, typename B>")
    w("  static MGRW_HD void external(const B& b, int h, ext<T>& w) {")
    for i, ip in enumerate(GLUON_PARTICLE[:ng]):
        out_flag = "true" if ip >= 2 else "false"
        w(f"    w.e{i} = gluon_pol<T>(b.g{i}, (h >> {next_ - 1 - ip}) & 1 ? 1 : -1, {out_flag});")
    w(f"    w.ub = ubar_out<T>(b.t, (h >> {next_ - 1 - 2}) & 1 ? 1 : -1);")
    w(f"    w.v = v_out<T>(b.tb, (h >> {next_ - 1 - 3}) & 1 ? 1 : -1);")
    w("  }")
    if vertex_kin:
        # programs reading their vertex momenta from the record take unit strong
        # couplings (every diagram carries g^NG); kappa enters through gk and,
        # at the top-vertex closures, through its powers gkp[n]
        w("  template <typename T> struct coup { T g, g2, gk; T gkp[NG + 1]; };")
        w("  template <typename T> static MGRW_HD coup<T> couplings(double gs, double gs2, double gk) {")
        w("    (void)gs2;")
        w("    const double kap = gk / gs;")
        w("    coup<T> c;")
        w("    c.g = T(1);")
        w("    c.g2 = T(1);")
        w("    c.gk = T(kap);")
        w("    double p = 1.0;")
        w("    for (int i = 0; i <= NG; ++i) { c.gkp[i] = T(p); p *= kap; }")
        w("    return c;")
        w("  }")
        w("  // NORM times g^(2 NG), the strong couplings the programs leave out")
        w("  static MGRW_HD double point_norm(double gs) {")
        w("    double f = NORM;")
        w("    for (int i = 0; i < NG; ++i) f *= gs * gs;")
        w("    return f;")
        w("  }")
    else:
        w("  template <typename T> struct coup { T g, g2, gk; };")
        w("  template <typename T> static MGRW_HD coup<T> couplings(double gs, double gs2, double gk) {")
        w("    return {T(gs), T(gs2), T(gk)};")
        w("  }")
        w("  static MGRW_HD double point_norm(double) { return NORM; }")
    w("  // Colour-flow amplitudes J of one helicity (common phase dropped).")
    w("  // k: the event's kin<T> (in registers or in LDS).")
    if body is not None:
        w("  static constexpr int NCHUNK = 1;")
        w("  template <typename T, typename KN>")
        w("  static MGRW_HD void amplitude(const ext<T>& w, const KN& k, const coup<T>& c, cx<T>* J) {")
        w("    for (int i = 0; i < K; ++i) J[i] = {T(0), T(0)};")
        for line in body:
            w("    " + line)
        w("  }")
    else:
        w(f"  static constexpr int NCHUNK = {len(part_ems)};")
        for ci, e in enumerate(part_ems):
            w(f"  // part {ci}: closing groups " + ", ".join(
                "leaf" if g == "leaf" else str(bits(g)) for g in parts[ci]))
            w("  template <typename T, typename KN>")
            w(f"  static MGRW_HD void amplitude_part{ci}(const ext<T>& w, const KN& k, const coup<T>& c, cx<T>* J) {{")
            for line in e.lines:
                w("    " + line)
            w("  }")
        w("  template <int C, typename T, typename KN>")
        w("  static MGRW_HD void amplitude_part(const ext<T>& w, const KN& k, const coup<T>& c, cx<T>* J) {")
        for ci in range(len(part_ems)):
            w(f"    {'if' if ci == 0 else 'else if'} constexpr (C == {ci}) amplitude_part{ci}<T>(w, k, c, J);")
        w("  }")
        w("  template <typename T, typename KN>")
        w("  static MGRW_HD void amplitude(const ext<T>& w, const KN& k, const coup<T>& c, cx<T>* J) {")
        w("    for (int i = 0; i < K; ++i) J[i] = {T(0), T(0)};")
        for ci in range(len(part_ems)):
            w(f"    amplitude_part{ci}<T>(w, k, c, J);")
        w("  }")
    if fr_ems:
        nch64, nfr = fp64_split
        w(f"  // Double-precision instance: {nch64} chunks of closing groups x {nfr} ranges of")
        w(f"  // {K // nfr} colour flows; amplitude_fr<C, R> adds chunk C's terms in flow range R")
        w("  // to J[0 .. KR-1] (flow R*KR + i in J[i]).")
        w(f"  static constexpr int NCHUNK64 = {nch64};")
        w(f"  static constexpr int NFR = {nfr};")
        w(f"  static constexpr int KR = {K // nfr};")
        for (c, r), (e, p) in sorted(fr_ems.items()):
            w(f"  // chunk {c} (closing groups " + ", ".join(
                "leaf" if g == "leaf" else str(bits(g)) for g in p) + f"), flows {r * (K // nfr)}..{(r + 1) * (K // nfr) - 1}")
            w("  template <typename T, typename KN>")
            w(f"  static MGRW_HD void amplitude_fr{c}_{r}(const ext<T>& w, const KN& k, const coup<T>& c, cx<T>* J) {{")
            for line in e.lines:
                w("    " + line)
            w("  }")
        w("  template <int C, int R, typename T, typename KN>")
        w("  static MGRW_HD void amplitude_fr(const ext<T>& w, const KN& k, const coup<T>& c, cx<T>* J) {")
        first = True
        for (c, r) in sorted(fr_ems):
            w(f"    {'if' if first else 'else if'} constexpr (C == {c} && R == {r}) amplitude_fr{c}_{r}<T>(w, k, c, J);")
            first = False
        w("  }")
    if body is not None:
        # kappa-polynomial form of the same diagrams: J split by power of kappa
        w("  // Same diagrams at unit couplings, J[(k-1)*K + w] collecting the diagrams")
        w("  // with k top-gluon vertices: J(g, kappa) = g^NG sum_k kappa^k J_k.")
        w("  // J: a pointer, or an accessor object with operator[] (entries kept partly")
        w("  // outside registers).")
        w("  template <typename T, typename KN, typename JA>")
        w("  static MGRW_HD void amplitude_kpoly(const ext<T>& w, const KN& k, const coup<T>& c, JA&& J) {")
        w("#if defined(__HIP_DEVICE_COMPILE__)")
        w("#pragma unroll")
        w("#endif")
        w("    for (int i = 0; i < NG * K; ++i) J[i] = {T(0), T(0)};")
        for line in kbody:
            w("    " + line)
        w("  }")
        w("  // Z = CF J (integer numerators), accumulated in T from inputs of type TI.")
        w("  template <typename T, typename TI>")
        w("  static MGRW_HD void colour_matvec(const cx<TI>* J, cx<T>* Z) {")
        for i in range(K):
            terms = [(num[i][j], j) for j in range(K) if num[i][j]]
            re = " + ".join(f"T({c}) * T(J[{j}].re)" for c, j in terms)
            im = " + ".join(f"T({c}) * T(J[{j}].im)" for c, j in terms)
            w(f"    Z[{i}] = {{{re}, {im}}};")
        w("  }")
        w("  template <typename T, typename TI>")
        w("  static MGRW_HD T re_dot(const cx<TI>* A, const cx<T>* Z) {")
        w("    T s = T(0);")
        w("    for (int i = 0; i < K; ++i) s = (s + T(A[i].re) * Z[i].re) + T(A[i].im) * Z[i].im;")
        w("    return s;")
        w("  }")
    w("  template <typename T>")
    w("  static MGRW_HD T colour_sum(const cx<T>* J) {")
    w("    T s = T(0);")
    for i in range(K):
        terms_re = [f"T({num[i][i]}) * J[{i}].re"]
        terms_im = [f"T({num[i][i]}) * J[{i}].im"]
        for j in range(i + 1, K):
            if num[i][j]:
                terms_re.append(f"T({2 * num[i][j]}) * J[{j}].re")
                terms_im.append(f"T({2 * num[i][j]}) * J[{j}].im")
        w(f"    {{ T zr = {terms_re[0]};")
        for t in terms_re[1:]:
            w(f"      zr = zr + {t};")
        w(f"      T zi = {terms_im[0]};")
        for t in terms_im[1:]:
            w(f"      zi = zi + {t};")
        w(f"      s = (s + zr * J[{i}].re) + zi * J[{i}].im; }}")
    w("    return s;")
    w("  }")
    w("  static constexpr int CF_NUM[K][K] = {")
    for row in num:
        w("    {" + ", ".join(str(x) for x in row) + "},")
    w("  };")
    if fr_ems:
        # the numerators as doubles, for the double-precision colour sum that
        # streams J from memory (row-major; CF is symmetric)
        w("  static constexpr double CF_DBL[K * K] = {")
        for row in num:
            w("    " + ", ".join(f"{x}.0" for x in row) + ",")
        w("  };")
    if chunks > 1:
        # colour matrix for the matrix cores: numerators padded to a multiple of
        # 32 and split exactly into two bfloat16 terms (bit patterns)
        kp = (K + 31) // 32 * 32
        hi, lo = bf16_split_table(num, kp)
        w("  static constexpr bool MFMA_COLOUR = true;")
        w(f"  static constexpr int KP = {kp};")
        w("  static constexpr unsigned short CF_BF16_HI[KP * KP] = {")
        for r in range(kp):
            w("    " + ", ".join(str(x) for x in hi[r * kp:(r + 1) * kp]) + ",")
        w("  };")
        w("  static constexpr unsigned short CF_BF16_LO[KP * KP] = {")
        for r in range(kp):
            w("    " + ", ".join(str(x) for x in lo[r * kp:(r + 1) * kp]) + ",")
        w("  };")
    w("};")
    w("}  // namespace mgrw")
    return "\n".join(out) + "\n", em
