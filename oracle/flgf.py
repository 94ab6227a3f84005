"""Oracle B: the Fast Lattice Green's Function method, step by step (plain CPU, FP64).

TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check and the CPU-baseline leg of
the benchmark may import this module; the product path never does.

This follows Sec. 3.1 ("Basic algorithm") in the paper's order and notation, with
numpy's FFT as the library primitive for the fast convolutions of Sec. 2.2:

  Step 0  pre-computation   khat^{P-Q} = FFT(k^{P-Q})                 (Eq. precomp)
  Step 1  upward pass       ftilde^P = sum_{Q in RegSupp(P)} Reg(ftilde^Q)   (Eq. alg_reg)
                            fhat^P = FFT(Pad(ftilde^P))                (Eq. alg_upfft)
  Step 2  level interactions uhat^P = sum_{Q in InflList(P)} Prod(fhat^Q, khat^{P-Q})
                                                                       (Eq. alg_mult)
  Step 3  downward pass     vtilde^P = Trunc(FFT^-1(uhat^P))           (Eq. alg_dwfft)
                            utilde^P = vtilde^P + Interp(utilde^{IntrpSupp(P)})
                                                                       (Eq. alg_interp)

Readings taken where the paper is silent or ambiguous (all listed in the design notes):
  * Block coordinates are shifted so the bounding-box minimum is 0; the level-1
    interval of block B has index B, and the parent of interval I is floor(I/2).
  * Interval I at level l >= 1 spans [I s_l, (I+1) s_l]^3 with s_l = n 2^(l-1); its
    p^3 nodes are x_{I,k} = I s_l + k h_l, h_l = s_l/(p-1) (one-node overlap on the
    + side, Sec. 4 footnote; p = n+1 gives the paper's own scheme).
  * Interpolation is Lagrange on the p nodes of an interval; with p > n_max = 10 each
    point uses only its n_max closest nodes (Sec. 2.5's hybrid p/h refinement; window
    start ceil(t - n_max/2), ties to the lower window, clamped to the interval).  Reg is
    the adjoint of Interp.
  * InflList: at level 0 the (up to) 27 blocks with |Q-P|_inf <= 1; at 1 <= l < L the
    children of the parent's neighbours with |Q-P|_inf >= 2; at the top level L all
    intervals with |Q-P|_inf >= 2.  L = min(levels, 1 + ceil(log2(extent))).
  * Separate source and evaluation blocks (B_s != B_e in Eq. bconv; the paper's Sec. 3.1
    takes them equal for brevity): both sets live on one lattice (shifted by the
    minimum over their union, extent of the union), the upward pass runs on the tree
    of the source blocks, the downward pass on the tree of the evaluation blocks, and
    every list pairs an evaluation interval P (target) with a source interval Q under
    the same geometric rules as above.
  * Kernel: level 0 uses the exact G.  Level l >= 1 uses G at lattice offsets with
    max|x_i| < R_LATTICE when the node spacing h_l is an integer, and the asymptotic
    expansion A^Q_FAR otherwise (the continuous part of Eq. dpsoln).
  * FFT convolution (Sec. 2.2, garbled indices): circular length M = 2m with m = n
    (level 0) or p (level >= 1); kernel value K(r) sits at index r mod M for
    r in [-(m-1), m-1], every other entry is 0; the output is entries [0, m).
  * A second non-oscillatory kernel (Sec. 5: the method applies to such LGFs): the LGF
    G_kappa of the screened operator L - kappa (kappa > 0).  It is used at every level
    from its integrated values (the method needs only kernel evaluations), so every node
    must lie on the lattice: (p - 1) must divide n, which makes h_l an integer at every
    level (p = n + 1 is the paper's scheme).
"""
import numpy as np

from . import lgf as _lgf

R_LATTICE = 32   # exact-G region for lattice kernels at levels >= 1
Q_FAR = 8        # terms of the asymptotic expansion used as the far kernel
N_MAX = 10       # most nodes one interpolation stencil uses (the paper's n_max)


# ----------------------------------------------------------------------------- layout / tree

def _as_blocks(blocks):
    """[N, 3] integer block coordinates (x, y, z); rejects empty sets and duplicates."""
    b = np.asarray(blocks, dtype=np.int64).reshape(-1, 3)
    if b.shape[0] == 0:
        raise ValueError("empty layout")
    if len({tuple(r) for r in b.tolist()}) != b.shape[0]:
        raise ValueError("duplicate blocks")
    return b


def normalize_blocks(blocks):
    """Shift block coordinates so the bounding-box minimum is 0 (translation-invariant
    tree anchoring)."""
    b = _as_blocks(blocks)
    return b - b.min(axis=0)


def full_depth(blocks):
    """1 + ceil(log2(extent)) with extent the largest bounding-box edge in blocks."""
    E = int(np.max(blocks.max(axis=0) + 1))
    d = 1
    while (1 << (d - 1)) < E:
        d += 1
    return d


class Tree:
    """Octree of intervals (Sec. 3.1) plus the lists RegSupp, IntrpSupp and InflList.

    Source side: `blocks`, `coords[l]`, `parent[l]` (the upward pass).  Evaluation side:
    `eval_blocks`, `coords_e[l]`, `parent_e[l]` (the downward pass); the same objects as
    the source side unless `eval_blocks` is given.  List entries are (target index on
    the evaluation side, source index on the source side, D = P - Q)."""

    def __init__(self, blocks, levels, eval_blocks=None):
        src = _as_blocks(blocks)
        ev = src if eval_blocks is None else _as_blocks(eval_blocks)
        lo = np.minimum(src.min(axis=0), ev.min(axis=0))
        self.blocks = src - lo
        self.eval_blocks = ev - lo
        fd = full_depth(np.vstack([self.blocks, self.eval_blocks]))
        self.L = fd if levels is None or levels <= 0 else min(int(levels), fd)
        self.coords, self.parent = self._levels(self.blocks)
        if eval_blocks is None:
            self.coords_e, self.parent_e = self.coords, self.parent
        else:
            self.coords_e, self.parent_e = self._levels(self.eval_blocks)
        # near-neighbour list at level 0: (target, source, D = P - Q)
        self.near = self._pairs(self.coords_e[1], self.coords[1], None, None, near=True)
        # interaction lists
        self.ilist = {}
        for l in range(1, self.L + 1):
            if l < self.L:
                pt = self.coords_e[l + 1][self.parent_e[l]]
                ps = self.coords[l + 1][self.parent[l]]
            else:
                pt = ps = None
            self.ilist[l] = self._pairs(self.coords_e[l], self.coords[l], pt, ps, near=False)

    def _levels(self, blocks):
        """coords[l] for l = 1..L (level-1 intervals are the blocks, same order) and
        parent[l][i] = index at level l + 1 of the parent of interval i."""
        coords = {1: blocks.copy()}
        parent = {}
        for l in range(1, self.L):
            par = coords[l] // 2
            uniq, inv = np.unique(par, axis=0, return_inverse=True)
            coords[l + 1] = uniq
            parent[l] = inv.reshape(-1)
        return coords, parent

    @staticmethod
    def _pairs(CT, CS, pt, ps, near):
        """All (P, Q, D = P - Q) of a list, by plain O(N^2) enumeration over targets CT
        and sources CS.
        near=True : |D|_inf <= 1 (near neighbours).
        near=False: |D|_inf >= 2, and if parent coordinates `pt` (of each target) and `ps`
                    (of each source) are given also |pt(P) - ps(Q)|_inf <= 1
                    (interaction list)."""
        tgt, src, off = [], [], []
        for i in range(CT.shape[0]):
            d = CT[i][None, :] - CS
            dinf = np.max(np.abs(d), axis=1)
            if near:
                mask = dinf <= 1
            else:
                mask = dinf >= 2
                if pt is not None:
                    mask &= np.max(np.abs(pt[i][None, :] - ps), axis=1) <= 1
            js = np.nonzero(mask)[0]
            tgt.extend([i] * len(js))
            src.extend(js.tolist())
            off.extend(d[js].tolist())
        return (np.asarray(tgt, dtype=np.int64), np.asarray(src, dtype=np.int64),
                np.asarray(off, dtype=np.int64).reshape(-1, 3))


# ----------------------------------------------------------------------------- interpolation

def stencil_start(p, t, nmax=N_MAX):
    """First node of the nmax consecutive nodes among 0..p-1 closest to t (Sec. 2.5: with
    more than n_max nodes only the n_max closest are used).  Every included node is at
    least as close as every excluded one when the window starts at ceil(t - nmax/2); a tie
    (t - nmax/2 an integer) goes to the lower window.  Clamped to the interval."""
    if p <= nmax:
        return 0
    return int(min(max(int(np.ceil(t - nmax / 2.0)), 0), p - nmax))


def lagrange(p, t, nmax=N_MAX):
    """phi_k(t) for the nodes 0..p-1, returned as [p, len(t)].  With p <= nmax this is the
    global Lagrange basis prod_{j != k} (t - j)/(k - j).  With p > nmax (hybrid p/h
    refinement, Sec. 2.5) each t uses the Lagrange basis of its nmax closest nodes, and
    phi_k(t) = 0 for the nodes outside that window."""
    t = np.atleast_1d(np.asarray(t, dtype=np.float64))
    out = np.zeros((p, t.size))
    for i, ti in enumerate(t.tolist()):
        lo = stencil_start(p, ti, nmax)
        win = range(lo, lo + min(p, nmax))
        for k in win:
            v = 1.0
            for j in win:
                if j != k:
                    v *= (ti - j) / (k - j)
            out[k, i] = v
    return out


def block_matrix(n, p, nmax=N_MAX):
    """A[k, j] = phi_k(j (p-1)/n): node k of a level-1 interval -> grid point j of its block."""
    return lagrange(p, np.arange(n) * (p - 1) / n, nmax)


def child_matrices(p, nmax=N_MAX):
    """C_c[m, k] = phi_m((c (p-1) + k)/2): parent node m -> node k of child c in {0, 1}."""
    return [lagrange(p, (c * (p - 1) + np.arange(p)) / 2.0, nmax) for c in (0, 1)]


def _apply3(Mz, My, Mx, X):
    """Y[b, a, c, d] = sum Mz[a, z] My[c, y] Mx[d, x] X[b, z, y, x]."""
    return np.einsum("az,cy,dx,bzyx->bacd", Mz, My, Mx, X, optimize=True)


def reg_block(A, f):
    """Reg from level 0 to level 1: ftilde = (A x A x A) f (Eq. kcprss1 in tensor form)."""
    return _apply3(A, A, A, f)


def interp_block(A, ut):
    """Interp from level 1 to level 0: u = (A^T x A^T x A^T) utilde (Eq. kcprss3)."""
    return _apply3(A.T, A.T, A.T, ut)


# ----------------------------------------------------------------------------- kernels

def level_geometry(n, p, l):
    """(s_l, h_l, lattice?) for level l >= 1."""
    s = n * 2 ** (l - 1)
    h = s / (p - 1)
    lattice = (s % (p - 1)) == 0
    return s, h, lattice


def kernel_values(x, lattice, kappa=0.0, h=1):
    """K_l at points x [..., 3] (float64) for a level >= 1 (see module docstring); with
    kappa > 0 the screened LGF at the lattice points x, multiples of the spacing h."""
    x = np.asarray(x, dtype=np.float64)
    if kappa > 0.0:
        if not lattice:
            raise ValueError("the screened kernel needs nodes on the lattice")
        return _lgf.lgf_lattice(np.rint(x).astype(np.int64), kappa, int(h))
    out = _lgf.asymptotic_values(x, Q_FAR)
    if lattice:
        xi = np.rint(x).astype(np.int64)
        near = np.max(np.abs(xi), axis=-1) < R_LATTICE
        if np.any(near):
            out[near] = _lgf.lgf(xi[near])
    return out


def kernel_block(D, m, origin_fn):
    """Real M^3 array (M = 2m), index [z, y, x]: K(D, r) at r mod M for r in
    [-(m-1), m-1]^3, zero elsewhere.  origin_fn(D, r) returns the kernel values."""
    M = 2 * m
    r1 = np.arange(-(m - 1), m)
    rz, ry, rx = np.meshgrid(r1, r1, r1, indexing="ij")
    r = np.stack([rx, ry, rz], axis=-1)  # (x, y, z) ordering of offsets
    vals = origin_fn(np.asarray(D), r)
    k = np.zeros((M, M, M))
    k[rz % M, ry % M, rx % M] = vals
    return k


def near_kernel_fn(n, kappa=0.0):
    def fn(D, r):
        return _lgf.lgf(D[None, None, None, :] * n + r, kappa)
    return fn


def far_kernel_fn(n, p, l, kappa=0.0):
    s, h, lattice = level_geometry(n, p, l)

    def fn(D, r):
        return kernel_values(D[None, None, None, :] * s + r * h, lattice, kappa, int(round(h)) if lattice else 1)
    return fn


# ----------------------------------------------------------------------------- FFT primitives

def pad_fft(x, M):
    """FFT(Pad(x)): zero-pad each m^3 block to M^3 and take the real-to-complex FFT."""
    return np.fft.rfftn(x, s=(M, M, M), axes=(1, 2, 3))


def ifft_trunc(uhat, M, m):
    """Trunc(FFT^-1(uhat)): inverse FFT, keep entries [0, m) per axis."""
    return np.fft.irfftn(uhat, s=(M, M, M), axes=(1, 2, 3))[:, :m, :m, :m]


# ----------------------------------------------------------------------------- the solver

class FLGF:
    """Plan + solve for u = G * f on a block layout, evaluated by the FLGF method.
    f lives on `blocks` (B_s); u is evaluated on `eval_blocks` (B_e), default B_s."""

    def __init__(self, blocks, n, p, levels, eval_blocks=None, kappa=0.0):
        self.n, self.p = int(n), int(p)
        self.kappa = _lgf._check_kappa(kappa)
        if self.kappa > 0.0 and self.n % (self.p - 1):
            raise ValueError("the screened kernel needs nodes on the lattice: (p - 1) must divide n")
        self.tree = Tree(blocks, levels, eval_blocks)
        self.A = block_matrix(self.n, self.p)
        self.C = child_matrices(self.p)
        # Step 0: pre-computation of every unique kernel spectrum used in Step 2
        M0 = 2 * self.n
        self.khat0 = {}
        for D in {tuple(d) for d in self.tree.near[2].tolist()}:
            self.khat0[D] = np.fft.rfftn(kernel_block(D, self.n, near_kernel_fn(self.n, self.kappa)))
        M1 = 2 * self.p
        self.khat = {}
        for l in range(1, self.tree.L + 1):
            fn = far_kernel_fn(self.n, self.p, l, self.kappa)
            for D in {tuple(d) for d in self.tree.ilist[l][2].tolist()}:
                self.khat[(l, D)] = np.fft.rfftn(kernel_block(D, self.p, fn))
        self.M0, self.M1 = M0, M1

    def _prod(self, fhat, pairs, khat_of, ntgt):
        """Step 2 for one level: uhat^P = sum_Q Prod(fhat^Q, khat^{P-Q}) for ntgt targets."""
        tgt, src, off = pairs
        uhat = np.zeros((ntgt,) + fhat.shape[1:], dtype=fhat.dtype)
        if tgt.size == 0:
            return uhat
        keys = [tuple(d) for d in off.tolist()]
        order = sorted(range(len(keys)), key=lambda i: keys[i])
        # group by offset: each target appears at most once per offset
        i = 0
        while i < len(order):
            D = keys[order[i]]
            j = i
            while j < len(order) and keys[order[j]] == D:
                j += 1
            sel = np.asarray(order[i:j])
            uhat[tgt[sel]] += fhat[src[sel]] * khat_of(D)[None]
            i = j
        return uhat

    def solve(self, f, return_levels=False):
        """f: [N_s, n, n, n] indexed [block, z, y, x] over the source blocks; returns u
        [N_e, n, n, n] over the evaluation blocks (the same blocks by default)."""
        t = self.tree
        n, p, L = self.n, self.p, t.L
        f = np.asarray(f, dtype=np.float64)
        # ---- Step 1: upward pass (on the source tree)
        ftil = {1: reg_block(self.A, f)}
        for l in range(1, L):
            par = t.parent[l]
            cpos = t.coords[l] - 2 * t.coords[l + 1][par]
            acc = np.zeros((t.coords[l + 1].shape[0], p, p, p))
            for c in range(8):
                cx, cy, cz = c & 1, (c >> 1) & 1, (c >> 2) & 1
                sel = np.nonzero((cpos[:, 0] == cx) & (cpos[:, 1] == cy) & (cpos[:, 2] == cz))[0]
                if sel.size == 0:
                    continue
                # Reg from child c: adjoint of Interp, i.e. apply C_c (parent m <- child k)
                contrib = _apply3(self.C[cz], self.C[cy], self.C[cx], ftil[l][sel])
                np.add.at(acc, par[sel], contrib)
            ftil[l + 1] = acc
        fhat0 = pad_fft(f, self.M0)
        fhat = {l: pad_fft(ftil[l], self.M1) for l in range(1, L + 1)}
        # ---- Step 2: level interactions
        uhat0 = self._prod(fhat0, t.near, lambda D: self.khat0[D], t.coords_e[1].shape[0])
        uhat = {l: self._prod(fhat[l], t.ilist[l], lambda D, l=l: self.khat[(l, D)], t.coords_e[l].shape[0])
                for l in range(1, L + 1)}
        # ---- Step 3: downward pass (on the evaluation tree)
        util, vtil = {}, {}
        for l in range(L, 0, -1):
            v = ifft_trunc(uhat[l], self.M1, p)
            vtil[l] = v.copy()
            if l < L:
                par = t.parent_e[l]
                cpos = t.coords_e[l] - 2 * t.coords_e[l + 1][par]
                for c in range(8):
                    cx, cy, cz = c & 1, (c >> 1) & 1, (c >> 2) & 1
                    sel = np.nonzero((cpos[:, 0] == cx) & (cpos[:, 1] == cy) & (cpos[:, 2] == cz))[0]
                    if sel.size == 0:
                        continue
                    v[sel] += _apply3(self.C[cz].T, self.C[cy].T, self.C[cx].T, util[l + 1][par[sel]])
            util[l] = v
        v0 = ifft_trunc(uhat0, self.M0, n)
        u = v0 + interp_block(self.A, util[1])
        if return_levels:
            return u, {"ftilde": ftil, "vnear": v0, "vtilde": vtil, "utilde": util}
        return u


def solve(blocks, f, n, p, levels, eval_blocks=None, kappa=0.0):
    return FLGF(blocks, n, p, levels, eval_blocks, kappa).solve(f)
