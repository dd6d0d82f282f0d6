"""The rank pass of the cell sort inside the fused push + deposit pass
(grpic_push_deposit_ranked, then grpic_sort_ranked) against the fused pass
followed by the separate sort (grpic_push_deposit, grpic_sort), through the C
ABI, in both precisions, on the library-function, long-series and
short-series kernels (48^2, 128^2, 512^2).  The slots are shuffled first, so
that a block of the pass holds up to 256 distinct cells (half its hash table),
and some are emptied.  Bars: the pushed states are the same bit for bit; the
sorted sets have the same cell sequence and the same particle states in each
cell bit for bit, and the same live count; the currents agree to the rounding
of the atomic additions' order.  A ranked sort whose ranks were consumed or
whose particle set changed since the ranked pass is refused.  At full size in
FP64 (C6 and C5, where the benchmark ranks inside the fused pass), the two
routes give the same live count and the same particle states per cell
(exact integer sums of the values' bit patterns)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

COLS = ["i1", "i2", "dx1", "dx2", "u1", "u2", "u3", "w", "phi", "tag"]


@pytest.fixture(scope="module")
def G():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2511_17701_amd import grpic
    torch.cuda.set_device(0)
    return grpic


def _context(G, w, prec):
    return G.Context(w.a, w.M, w.r_min, w.r_max, w.n_r, w.n_th, cfl=w.cfl, n_iter=w.n_iter,
                     small_angle=w.small_angle, charge_scale=1e-3, n_filter=w.n_filter,
                     n_absorb=w.n_absorb, precision=G.GRPIC_FP32 if prec == "fp32" else G.GRPIC_FP64)


def _rows(P, n):
    """Live rows of a cell-sorted set, ordered by cell and then by state."""
    cols = {k: P[k][:n].cpu().numpy() for k in COLS}
    bits = [cols[k].view(np.uint32 if cols[k].dtype.itemsize == 4 else np.uint64)
            if cols[k].dtype.kind == "f" else cols[k] for k in COLS]
    order = np.lexsort(bits[::-1])
    return {k: cols[k][order] for k in COLS}


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name,n", [("c1_64", 48), ("c3_2048", 128), ("c2_512", 512)])
def test_ranked_pass_and_sort_match_the_separate_sort(G, prec, name, n):
    import torch
    from paper_2511_17701_amd.workloads import WORKLOADS
    w = WORKLOADS[name].scaled(n, n)
    c = _context(G, w, prec)
    P = c.new_particles(w.n_particles)
    c.particles_init(P, w.n_pairs_total if w.ppc == 0 else 0, w.ppc, w.T, w.n_geo, w.seed)
    F = c.new_fields()
    c.fields_init_wald(F, w.B0)
    for _ in range(3):
        c.step(F, P, fused=True)
    gen = torch.Generator(device="cpu").manual_seed(11)
    perm = torch.randperm(w.n_particles, generator=gen).cuda()
    P = {k: v.index_select(0, perm).contiguous() for k, v in P.items()}
    P["tag"][::101] = 0
    P2 = {k: v.clone() for k, v in P.items()}
    F2 = F.clone()
    QA, QB = c.new_particles(w.n_particles), c.new_particles(w.n_particles)
    QB["tag"].fill_(5)  # the slots after the live ones must come back empty
    c.push_deposit(F, P)
    nA = c.sort(P, QA, count=True)
    c.push_deposit(F2, P2, ranked=True)
    nB = c.sort(P2, QB, count=True, ranked=True)
    torch.cuda.synchronize()
    for k in COLS + ["i2p", "dx1p", "dx2p"]:
        assert torch.equal(P[k], P2[k]), f"pushed state {k}"
    assert nA == nB and 0 < nB < w.n_particles
    assert (QB["tag"][nB:] == 0).all()
    a, b = _rows(QA, nA), _rows(QB, nB)
    key = b["i1"].astype(np.int64) * w.n_th + b["i2"]
    assert (np.diff(QB["i1"][:nB].cpu().numpy().astype(np.int64) * w.n_th
                    + QB["i2"][:nB].cpu().numpy()) >= 0).all()
    for k in COLS:
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)
    assert len(np.unique(key)) > 1
    tol = 1e-12 if prec == "fp64" else 1e-5
    for p in range(18, 21):
        s = float(F[p].abs().max())
        assert s > 0
        assert float((F[p].double() - F2[p].double()).abs().max()) <= tol * s, f"J plane {p}"
    # the ranks were consumed; a particle change in between ends their validity
    with pytest.raises(G.GrpicError):
        c.sort(P2, QB, ranked=True)
    c.push_deposit(F2, P2, ranked=True)
    c.push_deposit(F2, P2)
    with pytest.raises(G.GrpicError):
        c.sort(P2, QB, ranked=True)
    # a ranked pass on another set does not rank this one
    c.push_deposit(F, P, ranked=True)
    with pytest.raises(G.GrpicError):
        c.sort(P2, QB, ranked=True)
    del P, P2, QA, QB, F, F2
    torch.cuda.empty_cache()


def test_ranked_sort_of_an_empty_set(G):
    from paper_2511_17701_amd.workloads import WORKLOADS
    w = WORKLOADS["c1_64"].scaled(32, 32)
    c = _context(G, w, "fp64")
    F = c.new_fields()
    c.fields_init_wald(F, w.B0)
    E = c.new_particles(0)
    c.push_deposit(F, E, ranked=True)
    assert c.sort(E, c.new_particles(0), count=True, ranked=True) == 0


@pytest.mark.parametrize("name", ["c6_monopole", "c5_4096"])
def test_ranked_sort_full_size_fp64(G, name):
    """At full size in the form where the benchmark takes the ranked pass (FP64:
    C6, 2048^2 at 90 particles per cell = 3.77e8 particles, the paper's shape;
    C5, 4096^2 at 16), after 10 steps of motion: the ranked pass + ranked sort
    and the fused pass + separate sort give the same live count, both outputs
    are in cell order, and every cell holds the same particle states (per
    cell and array, the count and the integer sum of the values' bit patterns
    agree exactly)."""
    import torch
    from paper_2511_17701_amd.workloads import WORKLOADS
    w = WORKLOADS[name]
    c = G.Context(w.a, w.M, w.r_min, w.r_max, w.n_r, w.n_th, cfl=w.cfl, n_iter=w.n_iter,
                  small_angle=w.small_angle, charge_scale=w.charge_scale, n_filter=w.n_filter,
                  n_absorb=w.n_absorb, r0=w.r0, h0=w.h0, precision=G.GRPIC_FP64)
    F = c.new_fields()
    (c.fields_init_monopole if w.init == "monopole" else c.fields_init_wald)(F, w.B0)
    P = c.new_particles(w.n_particles)
    c.particles_init(P, w.n_pairs_total if w.ppc == 0 else 0, w.ppc, w.T, w.n_geo, w.seed)
    for _ in range(10):
        c.step(F, P, fused=True)
    P2 = {k: v.clone() for k, v in P.items()}
    F2 = F.clone()
    QA = c.new_particles(w.n_particles)
    c.push_deposit(F, P)
    nA = c.sort(P, QA, count=True)
    del P
    QB = c.new_particles(w.n_particles)
    c.push_deposit(F2, P2, ranked=True)
    nB = c.sort(P2, QB, count=True, ranked=True)
    del P2
    assert nA == nB and nB > 0.99 * w.n_particles
    ncell = w.n_r * w.n_th

    def summary(Q, n):
        cell = Q["i1"][:n].long() * w.n_th + Q["i2"][:n].long()
        assert bool((cell[1:] >= cell[:-1]).all()), "cell order"
        cnt = torch.zeros(ncell, dtype=torch.int64, device=cell.device).index_add_(
            0, cell, torch.ones_like(cell))
        sums = []
        for k in COLS:
            v = Q[k][:n]
            bits = (v.view(torch.int64) if v.dtype == torch.float64 else v.to(torch.int64))
            sums.append(torch.zeros(ncell, dtype=torch.int64, device=cell.device).index_add_(0, cell, bits))
        return cnt, sums

    ca, sa = summary(QA, nA)
    cb, sb = summary(QB, nB)
    assert torch.equal(ca, cb)
    for k, x, y in zip(COLS, sa, sb):
        assert torch.equal(x, y), k
    assert bool((QB["tag"][nB:] == 0).all())
    del QA, QB, F, F2
    torch.cuda.empty_cache()
