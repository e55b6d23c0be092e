"""The *_ws force entry points run in a caller-owned workspace, allocate
nothing, and give bit for bit the results of the allocating forms (which take
the same amount of stream-ordered memory per call).

Allocation is observed through the device's default memory pool, which
serves the allocating forms (hipMallocAsync): its high-water mark of used
bytes, reset before each call, stays 0 for a *_ws call and is at least the
queried size for the allocating form.
"""
import ctypes

import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

USED_MEM_HIGH = 0x8  # hipMemPoolAttrUsedMemHigh


@pytest.fixture(scope="module")
def sc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2602_20787_amd as m
    return m


@pytest.fixture(scope="module")
def pool():
    hip = ctypes.CDLL("libamdhip64.so")
    p = ctypes.c_void_p()
    assert hip.hipDeviceGetDefaultMemPool(ctypes.byref(p), 0) == 0

    class Pool:
        def reset(self):
            torch.cuda.synchronize()
            z = ctypes.c_uint64(0)
            assert hip.hipMemPoolSetAttribute(p, USED_MEM_HIGH, ctypes.byref(z)) == 0

        def high(self):
            torch.cuda.synchronize()
            v = ctypes.c_uint64(0)
            assert hip.hipMemPoolGetAttribute(p, USED_MEM_HIGH, ctypes.byref(v)) == 0
            return v.value
    return Pool()


def to_dev(p):
    d = torch.device("cuda:0")
    return (torch.from_numpy(p.pos).to(d), torch.from_numpy(p.mass).to(d),
            torch.from_numpy(p.eps).to(d))


def workspace(nbytes):
    # offset by 64 bytes from the allocation so that an unaligned base is exercised
    buf = torch.empty(nbytes + 64, dtype=torch.uint8, device="cuda:0")
    return buf[64:]


def check_same(plain, ws_out):
    for a, b in zip(plain, ws_out):
        if a is None:
            assert b is None
        else:
            assert torch.equal(a, b)


@pytest.mark.parametrize("N", [3000, 20000])
def test_exact_pairwise_in_a_workspace(sc, pool, N):
    p = synth.cylinder_load(N, seed=N)
    pos, m, e = to_dev(p)
    nb = sc.steps_cyl_forces_workspace(sc.STEPS_PATH_EXACT, N, 8, 0, sc.STEPS_SUM_PAIRWISE)
    assert nb > 32 * N
    print(f"[case] exact pairwise N={N} workspace {nb} B", flush=True)
    pool.reset()
    ref = sc.steps_cyl_forces(pos, m, e, p.L, 8)
    assert pool.high() >= nb - 256
    ws = workspace(nb)
    pool.reset()
    out = sc.steps_cyl_forces_ws(pos, m, e, p.L, 8, ws)
    assert pool.high() == 0
    check_same(ref, out)
    # the same call through the subset entry point's pairwise mode
    out2 = sc.steps_cyl_forces_ex_ws(pos, m, e, p.L, 8, ws, mode=sc.STEPS_SUM_PAIRWISE)
    check_same(ref, out2)


@pytest.mark.parametrize("n_targets", [100, 5000])
def test_per_target_and_f64_in_a_workspace(sc, pool, n_targets):
    p = synth.cylinder_load(9000, seed=3)
    pos, m, e = to_dev(p)
    t = torch.from_numpy(synth.target_sample(p.N, n_targets, seed=4)).cuda()
    nb = sc.steps_cyl_forces_workspace(sc.STEPS_PATH_EXACT, p.N, 8, n_targets, sc.STEPS_SUM_COMPENSATED)
    # lists of 4096 or more are ordered in the workspace, and these short
    # lists split the 9000 sources into chunks whose totals it holds
    assert nb >= 3 * 32 * n_targets
    ref = sc.steps_cyl_forces_ex(pos, m, e, p.L, 8, targets=t)
    ws = workspace(nb)
    pool.reset()
    out = sc.steps_cyl_forces_ex_ws(pos, m, e, p.L, 8, ws, targets=t)
    assert pool.high() == 0
    check_same(ref, out)
    nb64 = sc.steps_cyl_forces_workspace(sc.STEPS_PATH_F64, p.N, 8, n_targets, 0)
    assert nb64 > 0
    ref64 = sc.steps_cyl_forces_f64(pos, m, e, p.L, 8, targets=t)
    ws64 = workspace(nb64)
    pool.reset()
    out64 = sc.steps_cyl_forces_f64_ws(pos, m, e, p.L, 8, ws64, targets=t)
    assert pool.high() == 0
    check_same(ref64, out64)


def test_learned_and_table_in_a_workspace(sc, pool):
    p = synth.cylinder_load(5000, seed=8)
    pos, m, e = to_dev(p)
    net = sc.Mlp.create(synth.mlp_init(seed=21, out_gain=1.0))
    nb = sc.steps_cyl_forces_workspace(sc.STEPS_PATH_LEARNED, p.N, 0, 0, sc.STEPS_SUM_PAIRWISE)
    ref = sc.steps_cyl_forces_learned(pos, m, e, p.L, net)
    ws = workspace(nb)
    pool.reset()
    out = sc.steps_cyl_forces_learned_ws(pos, m, e, p.L, net, ws)
    assert pool.high() == 0
    check_same(ref, out)
    t = torch.arange(0, p.N, 1, dtype=torch.int64, device="cuda:0")
    nbl = sc.steps_cyl_forces_workspace(sc.STEPS_PATH_LEARNED, p.N, 0, p.N, sc.STEPS_SUM_COMPENSATED)
    refl = sc.steps_cyl_forces_learned_ex(pos, m, e, p.L, net, targets=t)
    wsl = workspace(nbl)
    pool.reset()
    outl = sc.steps_cyl_forces_learned_ex_ws(pos, m, e, p.L, net, wsl, targets=t)
    assert pool.high() == 0
    check_same(refl, outl)
    net.close()
    table = sc.CorrectionTable(32, 36, 6.4, 64)
    for targets in (None, t):
        n_t = 0 if targets is None else p.N
        nbt = sc.steps_cyl_forces_workspace(sc.STEPS_PATH_TABLE, p.N, 0, n_t, 0, table=table, order=1)
        reft = sc.steps_cyl_forces_table(pos, m, e, p.L, table, order=1, targets=targets)
        wst = workspace(nbt)
        pool.reset()
        outt = sc.steps_cyl_forces_table_ws(pos, m, e, p.L, table, wst, order=1, targets=targets)
        assert pool.high() == 0
        check_same(reft, outt)
    table.close()


def test_too_small_a_workspace_is_refused_before_any_launch(sc):
    p = synth.cylinder_load(4000, seed=9)
    pos, m, e = to_dev(p)
    nb = sc.steps_cyl_forces_workspace(sc.STEPS_PATH_EXACT, p.N, 8, 0, sc.STEPS_SUM_PAIRWISE)
    acc = torch.full((3, p.N), 7.0, dtype=torch.float32, device="cuda:0")
    with pytest.raises(sc.StepsError, match="workspace"):
        sc.steps_cyl_forces_ws(pos, m, e, p.L, 8, workspace(nb // 2), out_acc=acc, potential=False)
    torch.cuda.synchronize()
    assert torch.all(acc == 7.0)
