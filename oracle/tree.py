"""Binary tree of the TTN (paper Sec. 3.1), oracle side.

Reading used (the paper's tree has log2(N) - 1 layers with a two-tensor top):
a single root whose parent leg has dimension 1, so every one of the N - 1
internal nodes is a 3-leg tensor T[l, r, p].  The leaves are the sites in the
given leaf order; a k-leaf subtree splits into ceil(k/2) | floor(k/2).
Bond dimension of the link above a k-site subtree: min(m, d^k, d^(N-k))
(maximal possible dimension capped at m, Sec. 6.1.1 figure).
Node ids follow post-order (left subtree, right subtree, node): root = N - 2.
"""
from __future__ import annotations


class Tree:
    def __init__(self, leaf_order, m, d=2):
        self.leaf_order = list(leaf_order)
        self.N = N = len(leaf_order)
        self.m = m
        self.d = d
        self.children = []      # per node: [child_l, child_r]; child = ('n', id) | ('s', site)
        self.parent = []        # per node: parent id or -1
        self.sites_below = []   # per node: list of site ids in its subtree
        self.dims = []          # per node: (ml, mr, mp)
        self._build(0, N)
        self.root = len(self.children) - 1
        for n in range(self.n_nodes):
            for c in self.children[n]:
                if c[0] == 'n':
                    self.parent[c[1]] = n
        self.site_parent = {}
        for n in range(self.n_nodes):
            for side, c in enumerate(self.children[n]):
                if c[0] == 's':
                    self.site_parent[c[1]] = (n, side)
        self.below_set = [frozenset(s) for s in self.sites_below]

    def dim_of(self, k):
        if k == self.N:
            return 1
        return min(self.m, self.d ** k, self.d ** (self.N - k))

    def _build(self, lo, hi):
        k = hi - lo
        if k == 1:
            return ('s', self.leaf_order[lo])
        kl = (k + 1) // 2
        cl = self._build(lo, lo + kl)
        cr = self._build(lo + kl, hi)
        nid = len(self.children)
        self.children.append([cl, cr])
        self.parent.append(-1)
        self.sites_below.append(self.leaf_order[lo:hi])
        self.dims.append((self.dim_of(kl), self.dim_of(k - kl), self.dim_of(k)))
        return ('n', nid)

    @property
    def n_nodes(self):
        return len(self.children)

    def child_sites(self, n, side):
        c = self.children[n][side]
        return [c[1]] if c[0] == 's' else self.sites_below[c[1]]

    def regions(self, n):
        """(sites under left child, under right child, outside subtree(n))."""
        below = self.below_set[n]
        L = frozenset(self.child_sites(n, 0))
        R = frozenset(self.child_sites(n, 1))
        P = frozenset(s for s in range(self.N) if s not in below)
        return L, R, P

    def side_in_parent(self, n):
        q = self.parent[n]
        return 0 if self.children[q][0] == ('n', n) else 1

    def path(self, a, b):
        """Nodes from a to b inclusive along the tree."""
        anc_a = [a]
        while self.parent[anc_a[-1]] != -1:
            anc_a.append(self.parent[anc_a[-1]])
        anc_b = [b]
        while self.parent[anc_b[-1]] != -1:
            anc_b.append(self.parent[anc_b[-1]])
        set_b = set(anc_b)
        lca = next(x for x in anc_a if x in set_b)
        up = anc_a[:anc_a.index(lca) + 1]
        down = anc_b[:anc_b.index(lca)]
        return up + down[::-1]

    def post_order(self):
        return list(range(self.n_nodes))
