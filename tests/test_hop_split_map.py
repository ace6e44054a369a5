"""Host emulation of the LDS exchange of the hop with several threads per site
(paper_1701_00426_amd/csrc/hop_split.hip): which thread writes and reads which
entry of part[TPS-1][NR][3][SPB], and which thread stores which output entry, for
every field count a launch takes and 2 or 4 threads per site.

The live kernel: thread group q > 0 (whole waves, directions q*4/TPS ...) writes its
partial sums of every field to part[q-1]; after one barrier group 0 adds them in
the order q = 1, 2, 3 and stores every field.  The check is that every LDS access
is inside the array, every entry group 0 reads was written by exactly one thread
of the right group for the same (field, colour, site), and every output entry of
the chunk is stored exactly once.

It also emulates the epilogue variant that was removed after a wrong output entry
and a memory fault on the GPU (group q storing fields q, q + TPS, ... from totals
that group 0 leaves in LDS; its source was not kept), in its two plausible loop
forms, to record which of them stays inside the chunk.  No GPU is used.
"""
import itertools

import pytest

KBLOCK = 256
LDS_BUDGET = 48 * 1024  # kSplitLdsMax in kernels.hpp


def split_lds_bytes(elem, nr, tps):
    return (tps - 1) * nr * 3 * elem * (KBLOCK // tps)


def emulate_live(nr, tps):
    spb = KBLOCK // tps
    shape = (tps - 1, nr, 3, spb)
    writes, stores = {}, {}
    for tid in range(KBLOCK):
        q, l = tid // spb, tid % spb
        assert spb % 64 == 0  # every thread group is a whole number of waves
        if q > 0:
            for j in range(nr):
                for c in range(3):
                    idx = (q - 1, j, c, l)
                    assert all(0 <= idx[i] < shape[i] for i in range(4))
                    assert idx not in writes
                    writes[idx] = (q, j, c, l)
    for l in range(spb):  # group 0
        for r in range(tps - 1):
            for j in range(nr):
                for c in range(3):
                    idx = (r, j, c, l)
                    assert all(0 <= idx[i] < shape[i] for i in range(4))
                    assert writes[idx] == (r + 1, j, c, l)
        for j in range(nr):
            for c in range(3):
                assert (j, c, l) not in stores
                stores[(j, c, l)] = 0
    assert len(stores) == nr * 3 * spb
    assert len(writes) == (tps - 1) * nr * 3 * spb


def removed_variant_stores(nr, tps, guarded):
    """(field, colour, site) entries stored by group q in the removed epilogue:
    fields q, q + TPS, ... (guarded: only those below nr; unguarded: ceil(nr / TPS)
    of them whatever nr is)."""
    spb = KBLOCK // tps
    out = []
    for q in range(tps):
        count = -(-nr // tps)
        for k in range(count):
            j = q + k * tps
            if guarded and j >= nr:
                continue
            for c in range(3):
                for l in range(spb):
                    out.append((j, c, l))
    return out


@pytest.mark.parametrize("nr,tps", list(itertools.product((1, 2, 3, 4, 8), (2, 4))))
def test_live_split_exchange_exact_and_in_bounds(nr, tps):
    emulate_live(nr, tps)


def test_every_built_split_instantiation_fits_the_lds_budget():
    # the launcher builds 2 threads per site for every count, 4 where the budget allows
    built = []
    for elem in (8, 16):
        for nr in (1, 2, 3, 4, 8):
            assert split_lds_bytes(elem, nr, 2) <= LDS_BUDGET
            built.append((elem, nr, 2))
            if split_lds_bytes(elem, nr, 4) <= LDS_BUDGET:
                built.append((elem, nr, 4))
    assert (16, 8, 4) not in built            # 72 KiB: not built
    assert split_lds_bytes(16, 8, 4) == 73728


@pytest.mark.parametrize("nr,tps", list(itertools.product((1, 2, 3, 4, 8), (2, 4))))
def test_removed_variant_guarded_form_stores_the_chunk_exactly_once(nr, tps):
    st = removed_variant_stores(nr, tps, guarded=True)
    assert len(st) == len(set(st)) == nr * 3 * (KBLOCK // tps)
    assert all(j < nr for j, _, _ in st)


def test_removed_variant_unguarded_form_stores_past_the_chunk():
    """The unguarded loop stores fields nr .. TPS-1 when a chunk has fewer fields than
    threads per site.  Thirteen fields run as chunks of 8, 4 and 1; the last chunk
    starts at field 12, so with 4 threads per site groups 1-3 would store fields 13-15,
    beyond a 13-field output buffer: an out-of-bounds device store."""
    chunks = [8, 4, 1]
    beyond = []
    j0 = 0
    for nr in chunks:
        for j, _, _ in removed_variant_stores(nr, 4, guarded=False):
            if j0 + j >= 13:
                beyond.append(j0 + j)
        j0 += nr
    assert sorted(set(beyond)) == [13, 14, 15]
    # with 8 and 4 fields the unguarded form is exact
    for nr in (4, 8):
        st = removed_variant_stores(nr, 4, guarded=False)
        assert len(st) == len(set(st)) == nr * 3 * 64


def emulate_spread(nr, tps):
    """The spread epilogue: group q' writes its partial of every field j it does not
    own (owner o = j // (nr // tps)) to part[r][j] with r = q' if q' < o else q' - 1;
    after one barrier the owner adds the tps partials in the order q' = 0 .. tps-1
    (its own from registers) and stores field j.  Checks: every LDS access in bounds,
    no slot written twice, every slot the owner reads written by the right group for
    the same (field, colour, site), the same addition order as group 0 finishing
    every field, and every output entry stored exactly once."""
    assert nr % tps == 0
    spb = KBLOCK // tps
    k = nr // tps
    shape = (tps - 1, nr, 3, spb)
    writes, stores = {}, {}
    for tid in range(KBLOCK):
        q, l = tid // spb, tid % spb
        for j in range(nr):
            o = j // k
            if o == q:
                continue
            r = q if q < o else q - 1
            for c in range(3):
                idx = (r, j, c, l)
                assert all(0 <= idx[i] < shape[i] for i in range(4))
                assert idx not in writes
                writes[idx] = (q, j, c, l)
    for tid in range(KBLOCK):
        q, l = tid // spb, tid % spb
        for kk in range(k):
            j = q * k + kk
            for c in range(3):
                order = []
                for src in range(tps):
                    if src == q:
                        order.append(("own", q))
                    else:
                        idx = (src if src < q else src - 1, j, c, l)
                        assert all(0 <= idx[i] < shape[i] for i in range(4))
                        assert writes[idx] == (src, j, c, l)
                        order.append(("lds", src))
                assert [s for _, s in order] == list(range(tps))
                assert (j, c, l) not in stores
                stores[(j, c, l)] = q
    assert len(stores) == nr * 3 * spb
    assert len(writes) == (tps - 1) * nr * 3 * spb   # the same LDS as the live exchange


@pytest.mark.parametrize("nr,tps", [(2, 2), (4, 2), (8, 2), (4, 4), (8, 4)])
def test_spread_epilogue_exact_and_in_bounds(nr, tps):
    emulate_spread(nr, tps)


def layer_site(dims, G, pos):
    """Host copy of the layer order (kernels.hpp layer_site): position -> half index."""
    n0, n1, n2, n3 = dims
    L = n0 // 2 * n1
    lp, off = divmod(pos, L)
    gs = G * n2
    grp, r = divmod(lp, gs)
    x2, x3l = divmod(r, G)
    x3 = grp * G + x3l
    return (x2 + n2 * x3) * L + off


def layer_group_for(n3, want):
    """Host copy of capi.cpp layer_group_for: the largest divisor of N3 up to want."""
    if want <= 0:
        return 0
    for d in range(min(want, n3), 1, -1):
        if n3 % d == 0:
            return d
    return 0


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (4, 6, 8, 10), (6, 4, 2, 10), (32, 32, 32, 32),
                                  (24, 24, 24, 48), (16, 16, 16, 32), (10, 2, 4, 2)])
@pytest.mark.parametrize("want", [1, 2, 3, 4, 8, 16, 1024])
def test_layer_order_is_a_bijection_with_x3_fastest(dims, want):
    n0, n1, n2, n3 = dims
    vh = n0 * n1 * n2 * n3 // 2
    G = layer_group_for(n3, want)
    if G == 0:
        return  # half-index order
    assert n3 % G == 0
    hs = [layer_site(dims, G, p) for p in range(vh)]
    assert sorted(hs) == list(range(vh))
    L = n0 // 2 * n1
    # consecutive layers of one group and one x2 differ by one x3 plane
    for p in range(0, vh - L, L):
        lp = p // L
        if (lp % G) != G - 1:
            assert hs[p + L] - hs[p] == L * n2
