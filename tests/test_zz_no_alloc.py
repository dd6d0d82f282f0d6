"""grpic_sort_noalloc (the cell sort with the library's static scratch, for
callers that cannot allocate) against grpic_sort, through the C ABI.

The order of particles within one cell is unspecified for both, so what is
unique is compared bit for bit: the live count, the cell sequence of the
sorted slots, the multiset of particle states in every cell, and the emptied
tail.  Two calls in a row share the static array; the second sorts a smaller
set on a smaller grid (its counters must have been cleared).
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

STATE = ("i1", "i2", "dx1", "dx2", "u1", "u2", "u3", "w", "phi", "tag")


@pytest.fixture(scope="module")
def G():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2511_17701_amd import grpic
    torch.cuda.set_device(0)
    return grpic


def scrambled(G, n, n_pairs, precision, steps):
    """A loaded plasma (C1 recipe on an n x n grid) pushed a few steps in the
    Wald field so that cells and slots no longer agree, some slots emptied."""
    import torch
    from paper_2511_17701_amd.workloads import WORKLOADS
    w = WORKLOADS["c1_64"].scaled(n, n)
    ctx = G.Context(w.a, w.M, w.r_min, w.r_max, n, n, cfl=w.cfl, precision=precision)
    F = ctx.new_fields()
    ctx.fields_init_wald(F, w.B0)
    P = ctx.new_particles(2 * n_pairs)
    ctx.particles_init(P, n_pairs, 0, 1.0, 0, 4)
    for _ in range(steps):
        ctx.push(F, P)
    P["tag"][5::13] = 0
    perm = torch.randperm(2 * n_pairs, device=P["tag"].device, generator=None)
    for k in P:
        P[k] = P[k][perm].contiguous()
    torch.cuda.synchronize()
    return ctx, P


def canonical(P, n_live, n_th):
    """Live slots ordered by (cell, state): equal for any order within a cell."""
    h = {k: P[k].cpu().numpy() for k in STATE}
    live = {k: v[:n_live] for k, v in h.items()}
    key = live["i1"].astype(np.int64) * n_th + live["i2"]
    assert (np.diff(key) >= 0).all(), "sorted slots out of cell order"
    order = np.lexsort(tuple(live[k] for k in reversed(STATE[2:])) + (key,))
    return {k: v[order] for k, v in live.items()}, h["tag"][n_live:]


def check_same(G, ctx, P, n):
    import torch
    Qa = ctx.new_particles(P["tag"].numel())
    Qb = ctx.new_particles(P["tag"].numel())
    for Q in (Qa, Qb):               # destination tails hold garbage before the sort
        Q["tag"].fill_(9)
    n_a = ctx.sort(P, Qa, count=True)
    n_dev = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    ctx.sort_noalloc(P, Qb, n_live=n_dev)
    torch.cuda.synchronize()
    n_b = int(n_dev.item())
    assert n_b == n_a
    ca, ta = canonical(Qa, n_a, n)
    cb, tb = canonical(Qb, n_b, n)
    for k in STATE:
        np.testing.assert_array_equal(cb[k], ca[k], err_msg=k)
    assert (ta == 0).all() and (tb == 0).all()
    return n_a


def test_noalloc_sort_matches_sort_twice(G):
    """First call: FP64, 64^2 grid, 10^5 slots; second call: FP32, 32^2 grid,
    2 * 10^4 slots (a smaller input in the same static array)."""
    ctx1, P1 = scrambled(G, 64, 50_000, G.GRPIC_FP64, 3)
    n1 = check_same(G, ctx1, P1, 64)
    ctx2, P2 = scrambled(G, 32, 10_000, G.GRPIC_FP32, 2)
    n2 = check_same(G, ctx2, P2, 32)
    print(f"\n[sort_noalloc] live {n1} of 100000 (64^2), then {n2} of 20000 (32^2)")
    assert 0 < n2 < n1


def test_noalloc_sort_rejects_large_grids(G):
    """A grid of more than 2^24 cells is refused on the host; an empty set is
    sorted to an empty result with a live count of 0."""
    import torch
    ctx = G.Context(0.9, 1.0, 1.3, 20.0, 4097, 4096, dt=1e-3)
    P = ctx.new_particles(4)
    Q = ctx.new_particles(4)
    with pytest.raises(G.GrpicError, match="static sort scratch"):
        ctx.sort_noalloc(P, Q)
    ctx = G.Context(0.9, 1.0, 1.3, 20.0, 16, 16, dt=1e-3)
    n_dev = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    ctx.sort_noalloc(ctx.new_particles(0), ctx.new_particles(0), n_live=n_dev)
    torch.cuda.synchronize()
    assert int(n_dev.item()) == 0
