"""Host-side logic of the C-ABI library, on the CPU: argument checks that
return before anything is enqueued, and the batched problems' packing
(longest-first order, tile shapes, descriptor block).  Device pointers here
are aligned placeholder addresses that are never dereferenced."""
import ctypes
import os

import numpy as np
import pytest

from paper_2412_11079_amd import _lib

pytestmark = pytest.mark.skipif(not os.path.exists(_lib.LIB_PATH), reason="libuot.so not built")

FAKE = 0x7f0000000000       # 256-byte aligned placeholder device address


def _addr(k):
    return FAKE + 0x100000 * k


def _problem(n, m, dt=_lib.UOT_F32, k=0, eps=0.05, tau=1.0):
    p = _lib.Problem()
    p.n, p.m = n, m
    p.a, p.b = _addr(4 * k), _addr(4 * k + 1)
    p.k_dtype = dt
    p.K = _addr(4 * k + 2)
    es = {_lib.UOT_F64: 8, _lib.UOT_F32: 4, _lib.UOT_BF16: 2, _lib.UOT_FP8_E4M3: 1}[dt]
    p.ldk = (m + 63) // 64 * 64
    p.eps, p.tau, p.k_scale = eps, tau, 1.0
    return p


def _outputs(k):
    o = _lib.Outputs()
    base = FAKE + 0x40000000 + 0x100000 * k
    o.u, o.v, o.r, o.c, o.loss, o.info = (base + 0x1000 * i for i in range(6))
    return o


def _pack(ns, ms, dt=_lib.UOT_F32):
    count = len(ns)
    probs = (_lib.Problem * count)(*[_problem(n, m, dt, k) for k, (n, m) in enumerate(zip(ns, ms))])
    outs = (_lib.Outputs * count)(*[_outputs(k) for k in range(count)])
    opt = _lib.Options()
    opt.max_iter, opt.check_every, opt.fused = 10, 1, 1
    L = _lib.lib()
    nbytes = L.uot_batched_desc_bytes(count)
    host = (ctypes.c_uint8 * nbytes)()
    st = L.uot_batched_pack(probs, count, ctypes.byref(opt), outs, host, nbytes)
    return st, bytes(host), nbytes


def _words(blob, count):
    from paper_2412_11079_amd.batched import _DESC_WORDS
    return np.frombuffer(blob[:count * _DESC_WORDS * 8], dtype=np.int64).reshape(count, _DESC_WORDS)


def test_batched_pack_orders_longest_first_and_assigns_shapes():
    from paper_2412_11079_amd.batched import _DESC_INDEX_WORD, _DESC_SHAPE_WORD
    ns = [16, 2048, 700, 700, 1, 1500, 33]
    ms = [16, 2048, 1000, 1000, 2048, 257, 512]
    st, blob, nbytes = _pack(ns, ms)
    assert st == 0, _lib.lib().uot_last_error()
    w = _words(blob, len(ns))
    order = [int(x) for x in w[:, _DESC_INDEX_WORD]]
    # FP32 capacities: (rg 4, nc 1) 256, (4, 2) 512, (2, 2) 1024, (1, 2) 2048 columns
    expect = {16: 0, 257: 1, 512: 1, 1000: 4, 2048: 7}
    shapes = (w[:, _DESC_SHAPE_WORD] >> 32).astype(int)
    for q, i in enumerate(order):
        assert shapes[q] == expect[ms[i]], (ms[i], shapes[q])
    # estimated time: row steps ceil(n / rg) weighted by (3 + chunks per lane)
    rg_nc = {0: (4, 1), 1: (4, 2), 4: (2, 2), 7: (1, 2)}
    cost = [-(-ns[i] // rg_nc[expect[ms[i]]][0]) * (3 + rg_nc[expect[ms[i]]][1]) for i in order]
    assert cost == sorted(cost, reverse=True)
    assert order.index(2) < order.index(3)          # equal cost keeps the caller's order
    meta = _lib.BatchedMeta.from_buffer_copy(blob[nbytes - ctypes.sizeof(_lib.BatchedMeta):])
    assert meta.count == len(ns) and meta.k_dtype == _lib.UOT_F32 and meta.m_lds == 2048
    # without a device the resident workgroup count is unknown: nothing is split
    assert meta.items == len(ns) and meta.nsplit == 0 and meta.pool_bytes == 0


@pytest.mark.parametrize("dt,cap", [(_lib.UOT_F64, 2048), (_lib.UOT_F32, 2048), (_lib.UOT_BF16, 2048),
                                    (_lib.UOT_FP8_E4M3, 4096)])
def test_batched_row_capacity_per_dtype(dt, cap):
    assert _pack([8], [cap], dt)[0] == 0
    assert _pack([8], [cap + 1], dt)[0] == _lib.UOT_ERR_UNSUPPORTED


def test_batched_pack_rejects_bad_input():
    L = _lib.lib()
    probs = (_lib.Problem * 2)(_problem(10, 20, _lib.UOT_F32, 0), _problem(10, 20, _lib.UOT_F64, 1))
    outs = (_lib.Outputs * 2)(_outputs(0), _outputs(1))
    opt = _lib.Options()
    opt.max_iter, opt.check_every = 5, 1
    nb = L.uot_batched_desc_bytes(2)
    host = (ctypes.c_uint8 * nb)()
    assert L.uot_batched_pack(probs, 2, ctypes.byref(opt), outs, host, nb) == _lib.UOT_ERR_DTYPE
    probs[1] = _problem(10, 20, _lib.UOT_F32, 1)
    outs[1].loss = None
    assert L.uot_batched_pack(probs, 2, ctypes.byref(opt), outs, host, nb) == _lib.UOT_ERR_ARG
    outs[1] = _outputs(1)
    probs[0].K = _addr(0) + 4                                   # not 16-byte aligned
    assert L.uot_batched_pack(probs, 2, ctypes.byref(opt), outs, host, nb) == _lib.UOT_ERR_ALIGN
    probs[0] = _problem(10, 20, _lib.UOT_F32, 0)
    opt.absorb_log_threshold = 30.0
    assert L.uot_batched_pack(probs, 2, ctypes.byref(opt), outs, host, nb) == _lib.UOT_ERR_UNSUPPORTED
    opt.absorb_log_threshold = 0.0
    assert L.uot_batched_pack(probs, 2, ctypes.byref(opt), outs, host, nb - 1) == _lib.UOT_ERR_ARG
    assert L.uot_batched_pack(probs, 2, ctypes.byref(opt), outs, host, nb) == 0


def test_single_problem_argument_checks_happen_on_the_host():
    L = _lib.lib()
    opt = _lib.Options()
    opt.max_iter, opt.check_every, opt.fused = 5, 1, 1
    out = _outputs(0)

    def status(p, o=opt):
        return L.uot_sinkhorn(ctypes.byref(p), ctypes.byref(o), ctypes.byref(out), ctypes.c_void_p(FAKE), 1 << 20,
                              None)
    p = _problem(0, 10)
    assert status(p) == _lib.UOT_ERR_ARG
    p = _problem(10, 10, eps=0.0)
    assert status(p) == _lib.UOT_ERR_ARG
    p = _problem(10, 10, tau=-1.0)
    assert status(p) == _lib.UOT_ERR_ARG
    p = _problem(10, 10)
    p.K = _addr(2) + 8
    assert status(p) == _lib.UOT_ERR_ALIGN
    p = _problem(10, 10)
    p.k_dtype = 7
    assert status(p) == _lib.UOT_ERR_DTYPE
    p = _problem(10, 10)
    o2 = _lib.Options.from_buffer_copy(opt)
    o2.absorb_log_threshold = 30.0                              # absorption needs C
    assert status(p, o2) == _lib.UOT_ERR_ARG
    assert L.uot_sinkhorn_workspace_size(ctypes.byref(_problem(0, 10)), ctypes.byref(opt)) == 0
    msg = L.uot_last_error().decode()
    assert msg


def test_multi_and_plan_argument_checks_happen_on_the_host():
    L = _lib.lib()
    opt = _lib.Options()
    opt.max_iter, opt.check_every = 5, 1
    p = _problem(100, 100, _lib.UOT_F64)
    assert L.uot_sinkhorn_multi_workspace_size(ctypes.byref(p), 4, ctypes.byref(opt)) == 0
    assert L.uot_sinkhorn_multi(ctypes.byref(p), 4, _addr(10), _addr(11), ctypes.byref(opt), _addr(12), _addr(13),
                                _addr(14), _addr(15), ctypes.c_void_p(FAKE), 1 << 30, None) == _lib.UOT_ERR_DTYPE
    p = _problem(100, 100, _lib.UOT_BF16)
    assert L.uot_sinkhorn_multi_workspace_size(ctypes.byref(p), 0, ctypes.byref(opt)) == 0
    assert L.uot_sinkhorn_multi_workspace_size(ctypes.byref(p), 4, ctypes.byref(opt)) > 0
    opt.tol = 1e-6
    assert L.uot_sinkhorn_multi_workspace_size(ctypes.byref(p), 4, ctypes.byref(opt)) == 0
    q = _problem(10, 10)
    assert L.uot_plan(ctypes.byref(q), _addr(20), _addr(21), None, None, _addr(22), 10, _lib.UOT_BF16,
                      None) == _lib.UOT_ERR_DTYPE
    assert L.uot_plan(ctypes.byref(q), None, None, None, None, _addr(22), 10, _lib.UOT_F64, None) == _lib.UOT_ERR_ARG
    assert L.uot_plan(ctypes.byref(q), _addr(20), _addr(21), None, None, _addr(22), 5, _lib.UOT_F64,
                      None) == _lib.UOT_ERR_ARG


def test_strip_offsets_must_stay_below_2_gib():
    """A strip's loads use 32-bit byte offsets from its first row: a caller
    leading dimension that makes a strip (plus its prefetched rows) span
    2 GiB is refused on the host instead of wrapping."""
    L = _lib.lib()
    opt = _lib.Options()
    opt.max_iter, opt.check_every, opt.fused = 5, 1, 1
    p = _problem(300, 100)
    assert L.uot_sinkhorn_workspace_size(ctypes.byref(p), ctypes.byref(opt)) > 0
    p.ldk = 1 << 26                       # 256 MiB per FP32 row
    assert L.uot_sinkhorn_workspace_size(ctypes.byref(p), ctypes.byref(opt)) == 0
    out = _outputs(0)
    st = L.uot_sinkhorn(ctypes.byref(p), ctypes.byref(opt), ctypes.byref(out), ctypes.c_void_p(FAKE), 1 << 30, None)
    assert st == _lib.UOT_ERR_UNSUPPORTED
    assert b"2 GiB" in L.uot_last_error()
