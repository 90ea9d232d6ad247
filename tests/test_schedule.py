"""CPU checks of the create-time slot scheduler of the resident-weight kernel."""
import numpy as np
import pytest

import sdnn_inputs as gen

# Lanes served together by a 16-byte LDS read on gfx950 (measured with a lane-pair swap
# test): half-wave h = lane // 32 and parity of bits 2..4 of the lane give the unit.
UNITS = [[l for l in range(64) if 2 * (l >> 5) + (bin((l >> 2) & 7).count("1") & 1) == u] for u in range(4)]


@pytest.fixture(scope="module")
def P():
    import paper_2004_10908_amd as p
    return p


@pytest.mark.parametrize("N,L,seed", [(4096, 3, 1), (1024, 4, 2), (96, 2, 3), (2048, 2, 4)])
def test_schedule_invariants(P, N, L, seed):
    cfg = gen.tiny_config(N, L, 1, seed)
    idx = np.stack([gen.make_layer(cfg, l)[0] for l in range(L)])
    dmax = 44
    worst, ent, ln, steps = P.sdnn_schedule_host(idx, dmax)
    assert worst <= dmax
    nblk = (N + 63) // 64
    for l in range(L):
        seen = np.zeros(N, bool)
        for b in range(nblk):
            D = steps[l, b]
            lower = 32
            for lane in range(64):
                j = ln[l, 64 * b + lane]
                e = ent[l, 64 * b + lane, :D]
                real = e[(e >> 31) == 0]
                if j < 0:
                    assert real.size == 0
                    continue
                assert 64 * b <= j < 64 * b + 64 and not seen[j]
                seen[j] = True
                ks = (real & 31).astype(int)
                ids = (real >> 5).astype(int)
                assert sorted(ks) == list(range(32)), "each slot exactly once"
                assert np.array_equal(ids, idx[l, j, ks]), "entry id matches its slot"
                assert ((ent[l, 64 * b + lane, D:] >> 31) == 1).all()
            for u in UNITS:
                for s in range(D):
                    g = (ent[l, 64 * b + np.array(u), s] >> 5) % 16
                    assert len(set(g.tolist())) == 16, "a step of a unit must hit 16 bank groups"
            # balanced units need at least as many steps as their busiest bank group
            for u in UNITS:
                js = [ln[l, 64 * b + lane] for lane in u if ln[l, 64 * b + lane] >= 0]
                if js:
                    h = np.bincount((idx[l, js] % 16).ravel(), minlength=16)
                    lower = max(lower, h.max())
            assert lower <= D <= lower + 4
        assert seen.all()
    if N == 4096:
        assert steps.mean() < 39.5        # balancing keeps the padding near 20%


def test_schedule_rejects_bad_ids(P):
    idx = np.zeros((1, 64, 32), np.int32)
    idx[0, 0, 0] = 64
    with pytest.raises(P.SdnnError):
        P.sdnn_schedule_host(idx)


def _row_cost(idx, perm):
    """LDS passes of the one-row-tile kernel's reads, recomputed from the orders: per
    half-wave block of 32 consecutive neurons and step, the busiest bank's lane count
    (bank = input id mod 32)."""
    L, N, K = idx.shape
    order = np.take_along_axis(idx, perm.astype(np.int64), axis=2) % 32      # [L][N][step] banks
    cost = 0
    for l in range(L):
        for j0 in range(0, N, 32):
            blk = order[l, j0:j0 + 32]
            for s in range(K):
                cost += np.bincount(blk[:, s], minlength=32).max()
    return cost


@pytest.mark.parametrize("N,L,seed", [(2048, 2, 5), (2052, 1, 6), (4100, 1, 7)])
def test_row_schedule_orders(P, N, L, seed):
    """Bank-scheduled slot orders: each neuron reads each of its slots exactly once; the
    reported cost is the recomputed one; a full block costs at most 32 + K passes, K =
    max(max_b d_b - 32, 32 - min_b d_b) of its per-bank slot counts (the construction's
    bound), well under the ascending order's cost."""
    cfg = gen.tiny_config(N, L, 1, seed)
    idx = np.stack([gen.make_layer(cfg, l)[0] for l in range(L)])
    cost, perm = P.sdnn.sdnn_row_schedule_host(idx)
    assert (np.sort(perm, axis=2) == np.arange(32)).all(), "every slot exactly once per neuron"
    assert cost == _row_cost(idx, perm)
    ident = np.broadcast_to(np.arange(32, dtype=np.uint8), idx.shape)
    ascending = _row_cost(idx, ident)
    bound = 0
    for l in range(L):
        for j0 in range(0, N - N % 32, 32):
            d = np.bincount((idx[l, j0:j0 + 32] % 32).ravel(), minlength=32)
            bound += 32 + max(0, d.max() - 32, 32 - d.min())
    full = _row_cost(idx[:, : N - N % 32], perm[:, : N - N % 32])
    assert full <= bound
    assert cost < 0.5 * ascending, (cost, ascending)


def test_row_schedule_rejects_bad_ids(P):
    idx = np.zeros((1, 64, 32), np.int32)
    idx[0, 3, 7] = -1
    with pytest.raises(P.SdnnError):
        P.sdnn.sdnn_row_schedule_host(idx)
