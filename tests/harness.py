"""Shared helpers of the GPU parity tests: layout marshalling between the
oracle's per-leaf blocks ([ncomp][m+5][m+5]) and the library's state tensors,
and error measures.  No method arithmetic lives here."""
import numpy as np

import afsynth
import oracle
import paper_2205_07572_amd as af

KINDS = oracle.KINDS


def closed_masks(m, region=0):
    """Masks of the entries a step writes: interior cells and closed-square
    nodes (region 0), grown by one layer for region 1."""
    S1 = m + 5
    lo, hi = 2 - region, 2 + m + region
    mk = {}
    for kind in KINDS:
        a = np.zeros((S1, S1), bool)
        if kind == "avg":
            a[lo:hi, lo:hi] = True
        elif kind == "corner":
            a[lo:hi + 1, lo:hi + 1] = True
        elif kind == "xedge":
            a[lo:hi, lo:hi + 1] = True
        else:
            a[lo:hi + 1, lo:hi] = True
        mk[kind] = a
    return mk


def valid_masks(m):
    S1 = m + 5
    loc = np.arange(S1) - 2
    I, J = np.meshgrid(loc, loc)
    return {"avg": (I < m + 2) & (J < m + 2), "corner": np.ones_like(I, bool),
            "xedge": J < m + 2, "yedge": I < m + 2}


def rel_linf(got_blocks, ref_blocks, masks):
    """max |got - ref| / max |ref| over the masked entries of all blocks and
    kinds, per component."""
    nc = ref_blocks[0]["avg"].shape[0]
    num = np.zeros(nc)
    den = np.zeros(nc)
    for g, r in zip(got_blocks, ref_blocks):
        for kind in KINDS:
            mk = masks[kind] if isinstance(masks, dict) else masks[kind]
            for q in range(nc):
                num[q] = max(num[q], np.abs(g[kind][q][mk] - r[kind][q][mk]).max(initial=0.0))
                den[q] = max(den[q], np.abs(r[kind][q][mk]).max(initial=0.0))
    return num / np.maximum(den, 1e-300)


def oracle_blocks(h: "oracle.Hier"):
    return [h.get_block(k) for k in range(len(h.leaves()))]


def periodic_interior(blocks, leaves, m, n0):
    """Assemble owned DOFs of level-0 uniform blocks into periodic arrays."""
    nc = blocks[0]["avg"].shape[0]
    N = n0 * m
    out = {k: np.zeros((nc, N, N)) for k in KINDS}
    for b, (l, ix, iy) in zip(blocks, leaves):
        for k in KINDS:
            out[k][:, iy * m:(iy + 1) * m, ix * m:(ix + 1) * m] = b[k][:, 2:2 + m, 2:2 + m]
    return out


def make_problem(eq, prec, m, n0=1, lmax=0, lx=1.0, x0=0.0, a=1.0, b=0.5, c=1.0):
    return af.Problem(eq=eq, prec=prec, m=m, n0x=n0, n0y=n0, lmax=lmax, x0=x0, y0=x0, lx=lx, ly=lx,
                      a=a, b=b, c=c)


def leaf_blocks(prob, leaves, data, nq=6):
    out = []
    for (l, ix, iy) in leaves:
        dx, dy = prob.dx(l), prob.dy(l)
        out.append(afsynth.dofs_block(data, prob.m, 2, prob.x0 + ix * prob.m * dx, prob.y0 + iy * prob.m * dy,
                                      dx, dy, nq))
    return out
