"""Batch executor on the GPU: concurrent streams and graph replays give the
same results as the single calls, and the multi-instance shapes (32 uneven
2D SENSE problems plus a 128^3 kooshball) match the exact NUDFT on sampled
outputs.

The kernels are deterministic (no atomics), so a task run in a batch, eagerly
or from a graph, must equal the same call made alone bit for bit.
"""
import sys

import numpy as np
import pytest
import torch

from oracle import ndft
from paper_2111_02912_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL_NUFFT = 2e-5
TOL_JAC = 1e-4


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch.device("cuda", 0)


def _c(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex64)).to(dev)


def _f(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dev)


def _np(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


SMALL = dict(n2d=5, seed=4011, n_range=(24, 72), m_range=(500, 3000), coil_range=(1, 4),
             shape3d=(20, 16, 24), spokes3d=64, samples3d=48)


def _instances(dev, spec, seed0):
    from paper_2111_02912_amd.nufft import KbNufft
    out = []
    for i, inst in enumerate(W.multi_instance_case(**spec)):
        x, smaps, k = W.instance_data(inst, seed0 + 10 * i)
        plan = KbNufft(inst["N"], device=dev)
        plan.set_points(_f(inst["omega"], dev))
        out.append(dict(inst=inst, plan=plan, x=_c(x, dev), k=_c(k, dev),
                        smaps=_c(smaps, dev) if smaps is not None else None,
                        gimg=_c(W.complex_normal((1,) + tuple(inst["N"]), seed0 + 10 * i + 5), dev)))
    return out


def _all_op_tasks(items, dev):
    """Every task kind for every instance; outputs preallocated."""
    from paper_2111_02912_amd import batch as KB
    tasks, outs = [], []
    for it in items:
        p, C, M, D = it["plan"], it["inst"]["coils"], it["inst"]["omega"].shape[0], len(it["inst"]["N"])
        N = tuple(it["inst"]["N"])
        o = dict(y=torch.empty((1, C, M), dtype=torch.complex64, device=dev),
                 dwf=torch.empty((M, D), dtype=torch.float32, device=dev),
                 xa=torch.empty((1,) + N, dtype=torch.complex64, device=dev),
                 dwa=torch.empty((M, D), dtype=torch.float32, device=dev),
                 jxf=torch.empty((1,) + N, dtype=torch.complex64, device=dev),
                 jxa=torch.empty((1, C, M), dtype=torch.complex64, device=dev))
        s = it["smaps"]
        tasks += [KB.Task(p, KB.FORWARD, 1, C, it["x"], o["y"], s),
                  KB.Task(p, KB.JAC_OMEGA_FWD, 1, C, it["x"], o["dwf"], s, g=it["k"]),
                  KB.Task(p, KB.ADJOINT, 1, C, it["k"], o["xa"], s),
                  KB.Task(p, KB.JAC_OMEGA_ADJ, 1, C, it["k"], o["dwa"], s, g=it["gimg"]),
                  KB.Task(p, KB.JAC_X_FWD, 1, C, it["k"], o["jxf"], s),
                  KB.Task(p, KB.JAC_X_ADJ, 1, C, it["gimg"], o["jxa"], s)]
        outs.append(o)
    return tasks, outs


def _single_calls(it):
    from paper_2111_02912_amd import _lib
    p, s = it["plan"], it["smaps"]
    return dict(y=p.forward(it["x"], s), dwf=p.jac_omega_fwd(it["x"], it["k"], s),
                xa=p.adjoint(it["k"], s), dwa=p.jac_omega_adj(it["k"], it["gimg"], s),
                jxf=p.jac_x(_lib.KBN_OP_FORWARD, it["k"], s),
                jxa=p.jac_x(_lib.KBN_OP_ADJOINT, it["gimg"], s))


def _assert_equal(outs, refs, what):
    torch.cuda.synchronize()
    for i, (o, r) in enumerate(zip(outs, refs)):
        for k in r:
            assert torch.equal(o[k], r[k]), f"{what}: instance {i} output {k} differs"


@pytest.mark.parametrize("nstreams,fuse", [(1, False), (4, False), (1, True), (4, True)])
def test_batch_equals_single_calls(nstreams, fuse, dev):
    from paper_2111_02912_amd import batch as KB
    _say(f"batch eager + graph, nstreams={nstreams}, fused={fuse}")
    items = _instances(dev, SMALL, 5000)
    refs = [_single_calls(it) for it in items]
    tasks, outs = _all_op_tasks(items, dev)
    b = KB.KbnBatch(tasks, nstreams=nstreams, fuse=fuse)
    b.run()
    _assert_equal(outs, refs, "eager batch")
    for o in outs:
        for t in o.values():
            t.fill_(float("nan"))
    if fuse:
        # fused batches run eagerly: a second run rewrites every output, and
        # capture is refused on the host (the captured fused issue ended the
        # process in the graph runtime, so it stays switched off)
        b.run()
        _assert_equal(outs, refs, "second eager run")
        from paper_2111_02912_amd._lib import KbnError, KBN_ERR_UNSUPPORTED
        with pytest.raises(KbnError) as e:
            b.capture()
        assert e.value.code == KBN_ERR_UNSUPPORTED
        b.close()
        return
    b.capture()
    _assert_equal(outs, refs, "capture pass")
    for rep in range(3):
        for o in outs:  # eager work between replays: every replay must rewrite every output
            for t in o.values():
                t.fill_(float("nan"))
        torch.cuda.synchronize()
        b.launch()
        _assert_equal(outs, refs, f"replay {rep}")
    b.close()
    # and the single calls are right (forward and adjoint of two instances)
    for it, r in list(zip(items, refs))[-2:]:
        inst = it["inst"]
        s = _np(it["smaps"]) if it["smaps"] is not None else None
        y_ex = ndft.sense_forward(inst["omega"], _np(it["x"]), inst["N"], s)
        x_ex = ndft.sense_adjoint(inst["omega"], _np(it["k"]), inst["N"], s)
        assert ndft.rel_l2(_np(r["y"]), y_ex) < TOL_NUFFT
        assert ndft.rel_l2(_np(r["xa"]), x_ex) < TOL_NUFFT


def test_fused_batch_follows_new_points(dev):
    """A fused batch rebuilds its phases when a plan's points change (here
    with a different M) and still equals the single calls; on = 0 returns
    to per-task issue with the same results."""
    from paper_2111_02912_amd import _lib
    from paper_2111_02912_amd import batch as KB
    _say("fused batch after set_points")
    items = _instances(dev, dict(SMALL, n2d=3, shape3d=None), 5200)
    tasks, outs = _all_op_tasks(items, dev)
    b = KB.KbnBatch(tasks, nstreams=2, fuse=True)
    b.run()
    _assert_equal(outs, [_single_calls(it) for it in items], "fused, first points")
    held = items[0]["plan"].info()["device_bytes"]
    # new trajectory on plan 0 with more points: same output buffers cannot
    # hold them, so keep M and move the points instead
    it = items[0]
    om = W.uniform_random(it["inst"]["omega"].shape[0], len(it["inst"]["N"]), seed=5299)
    it["plan"].set_points(_f(om, dev))
    b.run()
    _assert_equal(outs, [_single_calls(it) for it in items], "fused, new points")
    assert items[0]["plan"].info()["device_bytes"] == held
    check = _lib.check
    check(_lib.lib().kbn_batch_fuse(b._h, 0), "kbn_batch_fuse")
    for o in outs:
        for t in o.values():
            t.fill_(float("nan"))
    b.run()
    _assert_equal(outs, [_single_calls(it) for it in items], "unfused again")
    assert items[0]["plan"].info()["device_bytes"] < held
    b.close()


def test_captured_plan_is_locked(dev):
    from paper_2111_02912_amd import batch as KB
    from paper_2111_02912_amd._lib import KbnError, KBN_ERR_UNSUPPORTED
    items = _instances(dev, dict(SMALL, n2d=2, shape3d=None), 5100)
    tasks, _ = _all_op_tasks(items, dev)
    b = KB.KbnBatch(tasks)
    b.capture()
    om = _f(items[0]["inst"]["omega"], dev)
    with pytest.raises(KbnError) as e:
        items[0]["plan"].set_points(om)
    assert e.value.code == KBN_ERR_UNSUPPORTED
    b.close()
    items[0]["plan"].set_points(om)


def test_multi_instance_shapes_sampled(dev):
    """Full-size instance mix, forward, adjoint and omega-Jacobian tasks
    from one graph (the task mix the batch benchmark times); sampled rows
    (forward, omega-gradient) and pixels (adjoint) of three instances, among
    them the 128^3 kooshball with M = 1,048,576."""
    from paper_2111_02912_amd import batch as KB
    _say("multi-instance full shapes")
    items = _instances(dev, {}, 6000)
    tasks, outs = [], []
    for it in items:
        inst = it["inst"]
        C, M, N = inst["coils"], inst["omega"].shape[0], tuple(inst["N"])
        y = torch.empty((1, C, M), dtype=torch.complex64, device=dev)
        xa = torch.empty((1,) + N, dtype=torch.complex64, device=dev)
        dw = torch.empty((M, len(N)), dtype=torch.float32, device=dev)
        tasks += [KB.Task(it["plan"], KB.FORWARD, 1, C, it["x"], y, it["smaps"]),
                  KB.Task(it["plan"], KB.JAC_OMEGA_FWD, 1, C, it["x"], dw, it["smaps"], g=it["k"]),
                  KB.Task(it["plan"], KB.ADJOINT, 1, C, it["k"], xa, it["smaps"])]
        outs.append((y, xa, dw))
    b = KB.KbnBatch(tasks)
    b.capture()
    b.launch()
    torch.cuda.synchronize()
    # the fused batch (one interpolation launch per phase and kernel shape,
    # run eagerly) gives the same bits as the per-task graph
    fused_outs = [tuple(torch.full_like(t, float("nan")) for t in o) for o in outs]
    ftasks = []
    for it, (y, xa, dw) in zip(items, fused_outs):
        C = it["inst"]["coils"]
        ftasks += [KB.Task(it["plan"], KB.FORWARD, 1, C, it["x"], y, it["smaps"]),
                   KB.Task(it["plan"], KB.JAC_OMEGA_FWD, 1, C, it["x"], dw, it["smaps"], g=it["k"]),
                   KB.Task(it["plan"], KB.ADJOINT, 1, C, it["k"], xa, it["smaps"])]
    fb = KB.KbnBatch(ftasks, fuse=True)
    fb.run()
    torch.cuda.synchronize()
    for i, (o, f) in enumerate(zip(outs, fused_outs)):
        for a, c, name in zip(o, f, ("y", "xa", "domega")):
            assert torch.equal(a, c), f"fused bundle: instance {i} {name} differs"
    fb.close()
    g = W.rng(6100)
    for i in (0, 5, len(items) - 1):
        it = items[i]
        inst = it["inst"]
        N, om = tuple(inst["N"]), inst["omega"]
        M = om.shape[0]
        s = _np(it["smaps"]) if it["smaps"] is not None else None
        rows = np.sort(g.choice(M, 64, replace=False))
        y_ex = ndft.sense_forward(om, _np(it["x"]), N, s, rows=rows)
        e_f = ndft.rel_l2(_np(outs[i][0])[:, :, rows], y_ex)
        pix = np.sort(g.choice(int(np.prod(N)), 32, replace=False))
        k = _np(it["k"])[0]
        xc = ndft.adjoint(om, k, N, pix=pix)  # [C, P]
        x_ex = (np.conj(s.reshape(s.shape[0], -1)[:, pix]) * xc).sum(0) if s is not None else xc[0]
        e_a = ndft.rel_l2(_np(outs[i][1]).reshape(-1)[pix], x_ex)
        dw_ex = ndft.jac_omega_fwd(om, _np(it["x"]), _np(it["k"]), N, s, rows=rows)
        e_j = ndft.rel_l2(_np(outs[i][2])[rows], dw_ex)
        _say(f"  instance {i} N={N} M={M} C={inst['coils']}: fwd {e_f:.2e} adj {e_a:.2e} "
             f"domega {e_j:.2e}")
        assert e_f < TOL_NUFFT and e_a < TOL_NUFFT and e_j < TOL_JAC
    b.close()
