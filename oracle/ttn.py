"""Isometric tree tensor network on the rotated Hamiltonian (oracle side).

Follows the paper step by step, in float64, with no fusion:

* Sec. 3.1: binary TTN of rank-3 tensors T[l, r, p]; every tensor except the
  isometry centre is an isometry toward the centre; QR decompositions move the
  centre (``_move_up`` / ``_move_down``), R is absorbed into the neighbour.
* Sec. 3.3.2: effective operators are built term by term; a term whose support
  lies inside one region of the centre is summed into that leg's operator, the
  others stay separate items passed to the matvec.
* Sec. 3.3.2 and 4.4.2: the generalised matvec contracts every item into the tensor in
  turn (``matvec``).
* Sec. 4 (steps 2-3): a DMRG sweep of single-tensor updates with the Lanczos
  eigensolver (``eigsolve``; the paper names Lanczos without details, read
  here as k = min(20, M) vectors from the current tensor, full
  reorthogonalisation, stop when beta_j <= 1e-14 max|alpha|, no restart).

Effective operators are kept per directed link and recomputed only for the
link the centre has just crossed.  For every link the oracle stores, besides
the summed local operator E, the renormalised image of every elementary
product operator (E_{o1 i1} x E_{o2 i2} x ...) on each site subset that a
crossing term has on that side.  Elementary products factorise across any
cut, so the recursion needs no decomposition; a term's renormalised factor is
the linear combination of these images with the term's own coefficients.
"""
from __future__ import annotations

import itertools

import numpy as np

from .tree import Tree
from .terms import rotate_all, compress_terms, realign, schmidt


def mode(A, x, j):
    """Mode-j product: (A x_j x)[.., i, ..] = sum_k A[i, k] x[.., k, ..].

    Written as one matrix product on a reshaped view of x (leg j first: A
    times x as a k x (rest) matrix; leg j last: x as a (rest) x k matrix times
    A^T; leg 1 of a 3-leg tensor: A times every x[a] slice), which is the same
    sum without transposed copies of x."""
    x = np.ascontiguousarray(x)
    if j == 0:
        return (A @ x.reshape(x.shape[0], -1)).reshape((A.shape[0],) + x.shape[1:])
    if j == x.ndim - 1:
        return (x.reshape(-1, x.shape[-1]) @ A.T).reshape(x.shape[:-1] + (A.shape[0],))
    if x.ndim == 3 and j == 1:
        return np.matmul(A, x)
    return np.moveaxis(np.tensordot(A, x, axes=(1, j)), 0, j)


def iso_qr(mat):
    """Householder QR (LAPACK) with the signs fixed so that diag(R) >= 0."""
    q, r = np.linalg.qr(mat)
    s = np.sign(np.diag(r))
    s[s == 0] = 1.0
    return q * s[None, :], r * s[:, None]


def _split_index(A, parts, d):
    """For an elementary index over the sorted site list A, the indices over
    each sub-list in ``parts``.  Index layout: out digits of the sites, then in
    digits (base d), first site most significant."""
    k = len(A)
    pos = {s: i for i, s in enumerate(A)}
    table = []
    for e in range(d ** (2 * k)):
        digits = []
        x = e
        for _ in range(2 * k):
            digits.append(x % d)
            x //= d
        digits = digits[::-1]
        outs, ins = digits[:k], digits[k:]
        sub = []
        for P in parts:
            idx = 0
            for s in P:
                idx = idx * d + outs[pos[s]]
            for s in P:
                idx = idx * d + ins[pos[s]]
            sub.append(idx)
        table.append(tuple(sub))
    return table


class Link:
    __slots__ = ("E", "R", "has_local")

    def __init__(self, E, R, has_local):
        self.E = E
        self.R = R
        self.has_local = has_local


class OracleTTN:
    def __init__(self, n_sites, d, m, leaf_order, terms, de_sites, de_u, raw_tensors,
                 krylov_k=20, structure_only=False, compress=False):
        self.tree = tr = Tree(leaf_order, m, d)
        assert tr.N == n_sites
        self.d = d
        self.krylov_k = krylov_k
        self.rterms = rotate_all(terms, de_sites, de_u, d)
        if compress:
            self.rterms = compress_terms(terms, self.rterms)
        self.supports = [frozenset(S) for S, _ in self.rterms]
        self.all_sites = frozenset(range(n_sites))
        self._needed = {}
        self.links = {}
        self.n_matvec = 0
        self.center = tr.root
        if structure_only:
            self.T = None
            return
        self.T = []
        for n, raw in enumerate(raw_tensors):
            ml, mr, mp = tr.dims[n]
            raw = np.asarray(raw, dtype=np.float64)
            assert raw.shape == (ml, mr, mp), (n, raw.shape, tr.dims[n])
            if n == tr.root:
                self.T.append(raw / np.linalg.norm(raw))
            else:
                q, _ = iso_qr(raw.reshape(ml * mr, mp))
                self.T.append(q.reshape(ml, mr, mp))
        for s in range(n_sites):
            self._compute_link(('up', ('s', s)))
        for n in range(tr.n_nodes):
            self._compute_link(('up', ('n', n)))

    def set_disentanglers(self, terms, de_sites, de_u, compress=False):
        """Replace the disentangler layer (Sec. 4, step 2 of each sweep): the
        rotated terms are rebuilt from the original ones, the tree tensors stay,
        and every link pointing toward the current centre is recomputed."""
        tr = self.tree
        self.rterms = rotate_all(terms, de_sites, de_u, self.d)
        if compress:
            self.rterms = compress_terms(terms, self.rterms)
        self.supports = [frozenset(S) for S, _ in self.rterms]
        self._needed = {}
        self.links = {}
        path = []
        x = self.center
        while x != -1:
            path.append(x)
            x = tr.parent[x]
        on_path = set(path)
        for s_ in range(tr.N):
            self._compute_link(('up', ('s', s_)))
        for n in range(tr.n_nodes):
            if n not in on_path:
                self._compute_link(('up', ('n', n)))
        for x in reversed(path[:-1]):
            self._compute_link(('down', x))

    # ------------------------------------------------------------ link bookkeeping
    def side(self, key):
        kind, who = key
        if kind == 'up':
            if who[0] == 's':
                return frozenset([who[1]])
            return self.tree.below_set[who[1]]
        return self.all_sites - self.tree.below_set[who]

    def needed_subsets(self, key):
        """Sorted site lists A = S' n side for every term crossing the link."""
        if key not in self._needed:
            side = self.side(key)
            out = set()
            for S in self.supports:
                inter = S & side
                if inter and not S <= side:
                    out.add(tuple(sorted(inter)))
            self._needed[key] = sorted(out)
        return self._needed[key]

    def _local_terms(self, side, part_a, part_b):
        """Terms inside ``side`` that meet both parts."""
        out = []
        for t, S in enumerate(self.supports):
            if S <= side and S & part_a and S & part_b:
                out.append(t)
        return out

    def _ren(self, link, A, vec):
        """Renormalised image of the operator with elementary coefficients
        ``vec`` over the site list A on ``link`` (identity if A is empty)."""
        if not A:
            return None
        return np.tensordot(vec, link.R[tuple(A)], axes=(0, 0))

    def _compute_link(self, key):
        tr = self.tree
        d = self.d
        kind, who = key
        side = self.side(key)
        need = self.needed_subsets(key)
        R = {}
        if kind == 'up' and who[0] == 's':
            s = who[1]
            E = np.zeros((d, d))
            has_local = False
            for t, S in enumerate(self.supports):
                if S == side:
                    E = E + self.rterms[t][1]
                    has_local = True
            for A in need:
                assert A == (s,)
                blocks = np.zeros((d * d, d, d))
                for o in range(d):
                    for i in range(d):
                        blocks[o * d + i, o, i] = 1.0
                R[A] = blocks
            self.links[key] = Link(E, R, has_local)
            return

        if kind == 'up':
            q = who[1]
            T = self.T[q]
            cl, cr = tr.children[q]
            kl, kr = ('up', cl), ('up', cr)
            Ll, Lr = self.links[kl], self.links[kr]
            sl, sr = self.side(kl), self.side(kr)

            def close(X):          # O[p, p'] = sum_{l r} T[l, r, p] X[l, r, p']
                return np.tensordot(T, X, axes=([0, 1], [0, 1]))

            def contract(Aop, Bop):
                X = T
                if Aop is not None:
                    X = mode(Aop, X, 0)
                if Bop is not None:
                    X = mode(Bop, X, 1)
                return close(X)

            E = close(mode(Ll.E, T, 0)) + close(mode(Lr.E, T, 1))
            has_local = Ll.has_local or Lr.has_local
            for t in self._local_terms(side, sl, sr):
                S, h = self.rterms[t]
                Al = sorted(self.supports[t] & sl)
                Ar = sorted(self.supports[t] & sr)
                sv, U, Vt = schmidt(realign(h, list(S), [Al, Ar], d))
                for k in range(len(sv)):
                    E = E + sv[k] * contract(self._ren(Ll, Al, U[:, k]),
                                             self._ren(Lr, Ar, Vt[k]))
                has_local = True
            for A in need:
                Al = [s for s in A if s in sl]
                Ar = [s for s in A if s in sr]
                table = _split_index(list(A), [Al, Ar], d)
                blocks = np.zeros((len(table), T.shape[2], T.shape[2]))
                cache_l = {}
                for e, (el, er) in enumerate(table):
                    if el not in cache_l:
                        cache_l[el] = mode(Ll.R[tuple(Al)][el], T, 0) if Al else T
                    X = cache_l[el]
                    if Ar:
                        X = mode(Lr.R[tuple(Ar)][er], X, 1)
                    blocks[e] = close(X)
                R[A] = blocks
            self.links[key] = Link(E, R, has_local)
            return

        # down link into node c from its parent q
        c = who
        q = tr.parent[c]
        T = self.T[q]
        cside = tr.side_in_parent(c)
        sib = tr.children[q][1 - cside]
        ks = ('up', sib)
        Ls = self.links[ks]
        ss = self.side(ks)
        if q == tr.root:
            Lp = None
            sp_ = frozenset()
        else:
            Lp = self.links[('down', q)]
            sp_ = self.side(('down', q))
        sib_leg = 1 - cside

        def close(X):          # O[c, c'] = sum over the other two legs
            other = [sib_leg, 2]
            return np.tensordot(T, X, axes=(other, other))

        def contract(Bop, Cop):
            X = T
            if Bop is not None:
                X = mode(Bop, X, sib_leg)
            if Cop is not None:
                X = mode(Cop, X, 2)
            return close(X)

        E = close(mode(Ls.E, T, sib_leg))
        has_local = Ls.has_local
        if Lp is not None:
            E = E + close(mode(Lp.E, T, 2))
            has_local = has_local or Lp.has_local
            for t in self._local_terms(side, ss, sp_):
                S, h = self.rterms[t]
                As = sorted(self.supports[t] & ss)
                Ap = sorted(self.supports[t] & sp_)
                sv, U, Vt = schmidt(realign(h, list(S), [As, Ap], d))
                for k in range(len(sv)):
                    E = E + sv[k] * contract(self._ren(Ls, As, U[:, k]),
                                             self._ren(Lp, Ap, Vt[k]))
                has_local = True
        for A in need:
            As = [s for s in A if s in ss]
            Ap = [s for s in A if s in sp_]
            table = _split_index(list(A), [As, Ap], d)
            mc = T.shape[cside]
            blocks = np.zeros((len(table), mc, mc))
            cache_s = {}
            for e, (es, ep) in enumerate(table):
                if es not in cache_s:
                    cache_s[es] = mode(Ls.R[tuple(As)][es], T, sib_leg) if As else T
                X = cache_s[es]
                if Ap:
                    X = mode(Lp.R[tuple(Ap)][ep], X, 2)
                blocks[e] = close(X)
            R[A] = blocks
        self.links[key] = Link(E, R, has_local)

    # ------------------------------------------------------------ effective Hamiltonian
    def node_links(self, n):
        tr = self.tree
        cl, cr = tr.children[n]
        Lp = None if n == tr.root else self.links[('down', n)]
        return self.links[('up', cl)], self.links[('up', cr)], Lp

    def node_regions(self, n):
        tr = self.tree
        cl, cr = tr.children[n]
        sl = self.side(('up', cl))
        sr = self.side(('up', cr))
        sp_ = frozenset() if n == tr.root else self.side(('down', n))
        return sl, sr, sp_

    def crossing_terms(self, n):
        sl, sr, sp_ = self.node_regions(n)
        out = []
        for t, S in enumerate(self.supports):
            k = (1 if S & sl else 0) + (1 if S & sr else 0) + (1 if S & sp_ else 0)
            if k >= 2:
                out.append(t)
        return out

    def prepare(self, n):
        """Collect the matvec items at node n (the centre).

        Each crossing term, realigned over its (l, r, p) site groups, is split
        first across (l r | p) and then each left factor across (l | r) by SVD
        (operator-Schmidt decompositions).  Returns (E_l, E_r, E_p, groups) with
        groups = [(W_coef, A_p or None, [(coef, A_l or None, A_r or None)])].
        """
        d = self.d
        Ll, Lr, Lp = self.node_links(n)
        sl, sr, sp_ = self.node_regions(n)
        groups = []
        for t in self.crossing_terms(n):
            S, h = self.rterms[t]
            Ss = self.supports[t]
            Al, Ar, Ap = sorted(Ss & sl), sorted(Ss & sr), sorted(Ss & sp_)
            t3 = realign(h, list(S), [Al, Ar, Ap], d)
            dl2, dr2, dp2 = t3.shape
            sv, Z, Vt = schmidt(t3.reshape(dl2 * dr2, dp2))
            for c in range(len(sv)):
                Op = self._ren(Lp, Ap, Vt[c]) if Ap else None
                if not Ap:
                    assert len(sv) == 1
                inner = []
                zs, U, Xt = schmidt(Z[:, c].reshape(dl2, dr2))
                for a in range(len(zs)):
                    # an empty group's factor is a scalar (+-1 after the SVD)
                    coef = zs[a] * (1.0 if Al else U[0, a]) * (1.0 if Ar else Xt[a, 0])
                    inner.append((coef, self._ren(Ll, Al, U[:, a]) if Al else None,
                                  self._ren(Lr, Ar, Xt[a]) if Ar else None))
                if not Ap:
                    # the p-side factor is the scalar Vt[0, 0]
                    groups.append((sv[c] * Vt[c, 0], None, inner))
                else:
                    groups.append((sv[c], Op, inner))
        El, Er = Ll.E, Lr.E
        Ep = Lp.E if Lp is not None else np.zeros((1, 1))
        return El, Er, Ep, groups

    def matvec(self, n, x, prep=None):
        """y = H_eff(n) x for x of shape (ml, mr, mp)."""
        El, Er, Ep, groups = prep if prep is not None else self.prepare(n)
        y = mode(El, x, 0) + mode(Er, x, 1) + mode(Ep, x, 2)
        for wc, Op, inner in groups:
            W = mode(Op, x, 2) if Op is not None else x
            for c, Al, Ar in inner:
                V = W
                if Ar is not None:
                    V = mode(Ar, V, 1)
                if Al is not None:
                    V = mode(Al, V, 0)
                y += (wc * c) * V
        self.n_matvec += 1
        return y

    # ------------------------------------------------------------ local eigensolver
    def eigsolve(self, n):
        """Lowest eigenpair of H_eff(n), warm start from T_n.  Plain Lanczos:
        k = min(krylov_k, M) matvecs, three-term recurrence followed by two
        passes of classical Gram-Schmidt against all previous vectors, stop when
        beta_j <= 1e-14 max|alpha|; lowest eigenpair of the tridiagonal matrix;
        Ritz vector normalised; its sign (a gauge) is fixed by making the first
        component of the tridiagonal eigenvector with magnitude >= 1e-8 of the
        largest one positive (the overlap with the start vector when that is
        not negligible).  The Ritz vector replaces T_n."""
        shape = self.T[n].shape
        M = int(np.prod(shape))
        k = min(self.krylov_k, M)
        prep = self.prepare(n)
        v = self.T[n].reshape(-1).copy()
        v /= np.linalg.norm(v)
        V = [v]
        alphas, betas = [], []
        for j in range(k):
            w = self.matvec(n, V[j].reshape(shape), prep).reshape(-1)
            a = float(V[j] @ w)
            alphas.append(a)
            if j == k - 1:
                break
            w = w - a * V[j]
            if j > 0:
                w = w - betas[j - 1] * V[j - 1]
            Vm = np.array(V)
            for _ in range(2):
                w = w - Vm.T @ (Vm @ w)
            b = float(np.linalg.norm(w))
            if b <= 1e-14 * max(abs(x) for x in alphas):
                break
            betas.append(b)
            V.append(w / b)
        ke = len(alphas)
        Tm = np.diag(alphas) + np.diag(betas[:ke - 1], 1) + np.diag(betas[:ke - 1], -1)
        evals, evecs = np.linalg.eigh(Tm)
        theta = float(evals[0])
        y = evecs[:, 0]
        nz = np.flatnonzero(np.abs(y) >= 1e-8 * np.abs(y).max())
        if y[nz[0]] < 0:
            y = -y
        x = np.array(V[:ke]).T @ y
        x /= np.linalg.norm(x)
        self.T[n] = x.reshape(shape)
        self.last_krylov = ke
        return theta

    # ------------------------------------------------------------ isometrisation
    def _move_up(self, n):
        tr = self.tree
        q = tr.parent[n]
        ml, mr, mp = self.T[n].shape
        Q, R = iso_qr(self.T[n].reshape(ml * mr, mp))
        self.T[n] = Q.reshape(ml, mr, Q.shape[1])
        self.T[q] = mode(R, self.T[q], tr.side_in_parent(n))
        self.center = q
        self._compute_link(('up', ('n', n)))

    def _move_down(self, q, c):
        tr = self.tree
        leg = tr.side_in_parent(c)
        Tq = np.moveaxis(self.T[q], leg, 2)
        sh = Tq.shape
        Q, R = iso_qr(Tq.reshape(sh[0] * sh[1], sh[2]))
        self.T[q] = np.moveaxis(Q.reshape(sh[0], sh[1], Q.shape[1]), 2, leg)
        self.T[c] = mode(R, self.T[c], 2)
        self.center = c
        self._compute_link(('down', c))

    def move_center(self, n):
        path = self.tree.path(self.center, n)
        for a, b in zip(path[:-1], path[1:]):
            if self.tree.parent[a] == b:
                self._move_up(a)
            else:
                self._move_down(a, b)

    def sweep(self):
        """One sweep: post-order visit of every node (left subtree, right
        subtree, node), centre moved link by link, eigensolve at each node.
        Returns theta at the last node (the root)."""
        theta = None
        for n in self.tree.post_order():
            self.move_center(n)
            theta = self.eigsolve(n)
        return theta

    # ------------------------------------------------------------ cost model
    def flops(self, n):
        """Algorithmic flops of one matvec at node n: summed local legs 2 m_j M;
        two-leg terms 2 M t (m_a + m_b); three-leg terms as the cheapest chain
        2 M (t_a m_a + t_a t_c m_b + t_c m_c); t = operator-Schmidt ranks."""
        ml, mr, mp = self.tree.dims[n]
        M = ml * mr * mp
        dims = (ml, mr, mp)
        regs = self.node_regions(n)
        tr = self.tree
        F = 0
        for j in range(3):
            if j == 2 and n == tr.root:
                continue
            if any(S <= regs[j] for S in self.supports):
                F += 2 * dims[j] * M
        for t in self.crossing_terms(n):
            S, h = self.rterms[t]
            parts = [sorted(self.supports[t] & r) for r in regs]
            present = [j for j in range(3) if parts[j]]
            if len(present) == 2:
                a, b = present
                mat = realign(h, list(S), [parts[a], parts[b]], self.d)
                tb = len(schmidt(mat)[0])
                F += 2 * M * tb * (dims[a] + dims[b])
            else:
                ranks = []
                for j in range(3):
                    rest = [s for k in range(3) if k != j for s in parts[k]]
                    mat = realign(h, list(S), [parts[j], rest], self.d)
                    ranks.append(len(schmidt(mat)[0]))
                best = None
                for b in range(3):
                    a, c = [j for j in range(3) if j != b]
                    cost = 2 * M * (ranks[a] * dims[a] + ranks[a] * ranks[c] * dims[b]
                                    + ranks[c] * dims[c])
                    best = cost if best is None else min(best, cost)
                F += best
        return F


def full_state(tree, T, d=2):
    """The TTN contracted into a 2^N vector (site 0 most significant)."""
    def rec(child):
        if child[0] == 's':
            return np.eye(d)
        n = child[1]
        cl, cr = tree.children[n]
        Pl, Pr = rec(cl), rec(cr)
        X = np.einsum('al,br,lrp->abp', Pl, Pr, T[n])
        return X.reshape(Pl.shape[0] * Pr.shape[0], T[n].shape[2])
    psi = rec(('n', tree.root)).reshape(-1)
    N = tree.N
    t = psi.reshape([d] * N)
    pos = {s: i for i, s in enumerate(tree.leaf_order)}
    t = t.transpose([pos[s] for s in range(N)])
    return t.reshape(-1)


def embedding_columns(ttn, n, d=2):
    """P_n: columns are the full states obtained by replacing the centre tensor
    T_n with each unit tensor (node n must be the isometry centre)."""
    shape = ttn.T[n].shape
    M = int(np.prod(shape))
    keep = ttn.T[n]
    cols = []
    for k in range(M):
        e = np.zeros(M)
        e[k] = 1.0
        ttn.T[n] = e.reshape(shape)
        cols.append(full_state(ttn.tree, ttn.T, d))
    ttn.T[n] = keep
    return np.array(cols).T
