"""Bit-exact checks of the integer work of the block sort (the counting sort
that groups the particles by 4^3-node grid block for the transfers): every
particle appears once, each occupied block's segment holds exactly the
particles whose stencil base lies in that block, and the block counts equal
a numpy histogram of the keys computed here from the positions."""
import numpy as np
import pytest

from paper_2303_02346_amd import scenes

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)


def spread3(v):
    """Bit i of v moved to bit 3 i."""
    out = np.zeros_like(v, dtype=np.uint64)
    for i in range(11):
        out |= ((v.astype(np.uint64) >> np.uint64(i)) & np.uint64(1)) << np.uint64(3 * i)
    return out


def block_keys(x, n_grid, scene):
    """Key of the block of each particle's stencil base floor(x/dx - 1/2):
    (scene << 3 kb) | Morton interleave of the block coordinates, x bits
    above y bits above z bits, kb bits per axis for ceil(n_grid / 4)
    blocks.  Positions go through FP32 as on the GPU."""
    xf = np.asarray(x, np.float32)
    base = np.floor(xf * np.float32(n_grid) - np.float32(0.5)).astype(np.int64)
    b = base >> 2
    nb = (n_grid + 3) // 4
    kb = 0
    while (1 << kb) < nb:
        kb += 1
    m = (spread3(b[:, 0]) << np.uint64(2)) | (spread3(b[:, 1]) << np.uint64(1)) | spread3(b[:, 2])
    return ((np.asarray(scene, np.uint64) << np.uint64(3 * kb)) | m).astype(np.uint64)


def check_sort(sim, x, n_grid, scene, which=0):
    """which = 0: the import of a call, whose block list gives the blocks of
    more than 256 particles first; which = 2: the sort of the adjoint's
    recompute, whose block list must be in increasing key order (the scan
    over all keys)."""
    ids, keys, lst = sim.sort_snapshot(which)
    N = x.shape[0]
    # every particle exactly once
    assert np.array_equal(np.sort(ids.astype(np.int64)), np.arange(N))
    # the sorted keys are the keys of the sorted particles
    ref = block_keys(x, n_grid, scene)
    assert np.array_equal(keys.astype(np.uint64), ref[ids])
    # the list partitions [0, N) into one segment per occupied key
    lk, lo, cnt = lst[:, 0].astype(np.int64), lst[:, 1].astype(np.int64), lst[:, 2].astype(np.int64)
    order = np.argsort(lo)
    assert lo[order][0] == 0 and np.array_equal(lo[order][1:], (lo + cnt)[order][:-1]) and (lo + cnt).max() == N
    assert (cnt > 0).all() and len(np.unique(lk)) == len(lk)
    if which == 2:
        assert (np.diff(lk) > 0).all()
    else:
        # longest first: the blocks of more than one 256-particle chunk are
        # listed before those of one
        big = cnt > 256
        assert not (big[1:] & ~big[:-1]).any()
    for k, o, c in zip(lk, lo, cnt):
        assert (keys[o:o + c] == k).all()
    # counts equal the histogram of the keys
    uk, uc = np.unique(ref, return_counts=True)
    h = dict(zip(uk.tolist(), uc.tolist()))
    assert len(h) == len(lk) and all(h[int(k)] == int(c) for k, c in zip(lk, cnt))
    return len(lk)


def test_sort_config2_bit_exact():
    from paper_2303_02346_amd.sim import Simulator
    sc = scenes.config2()
    sim = Simulator(sc)
    nl = check_sort(sim, sc.x, sc.n_grid, np.zeros(sc.n, np.int64))
    say(f"  config 2: {sc.n} particles in {nl} blocks, ids, keys, segments and counts exact")
    check_sort(sim, sc.x, sc.n_grid, np.zeros(sc.n, np.int64), which=2)
    say("  the same with the blocks in key order")
    # the buffer left by fused steps (sorted by the fused kernel's own key
    # counting and scans) still holds every particle once
    sim.step(20)
    ids = sim.sort_snapshot(1)
    assert np.array_equal(np.sort(ids.astype(np.int64)), np.arange(sc.n))
    # and a sort of the advanced state is exact again
    check_sort(sim, sim.positions(), sc.n_grid, np.zeros(sc.n, np.int64))


def test_sort_config4_full_bit_exact():
    """The 64-scene batch (3.8M particles, 6-bit scene prefix in the keys)."""
    from paper_2303_02346_amd.sim import Simulator
    scs = scenes.config4(steps=4)
    sim = Simulator(scs)
    x = np.concatenate([sc.x for sc in scs])
    scene = np.concatenate([np.full(sc.n, s) for s, sc in enumerate(scs)])
    nl = check_sort(sim, x, scs[0].n_grid, scene)
    say(f"  config 4: {x.shape[0]} particles of {len(scs)} scenes in {nl} blocks, exact")
    check_sort(sim, x, scs[0].n_grid, scene, which=2)
    say("  the same with the blocks in key order")
    sim.step(4)
    ids = sim.sort_snapshot(1)
    assert np.array_equal(np.sort(ids.astype(np.int64)), np.arange(x.shape[0]))
