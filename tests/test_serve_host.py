"""Host-side behaviour of the serving form that needs no device: request
validation, admission limits checked at submission, and the queued-state
operations (poll, cancel, stop) of a server started paused, which admits
nothing and so never touches the GPU."""
import numpy as np
import pytest

import graphgen as gg


@pytest.fixture
def hb():
    import paper_1308_2144_amd as hb

    return hb


def test_submission_checks(hb):
    off, idx = gg.directed_cycle(10)
    with hb.Server(start_paused=True, budget_bytes=1 << 20, max_nodes=4096, max_arcs=1000) as srv:
        for b in (3, 9):
            with pytest.raises(hb.HBError) as e:
                srv.submit(off, idx, b, 1)
            assert e.value.status == hb.HB_EINVAL and "log2m" in str(e.value)
        bad = idx.copy()
        bad[3] = 10                                   # index outside [0, n)
        with pytest.raises(hb.HBError) as e:
            srv.submit(off, bad, 4, 1)
        assert e.value.status == hb.HB_EINVAL
        bad_off = off.copy()
        bad_off[5], bad_off[6] = bad_off[6], bad_off[5]   # not monotone
        with pytest.raises(hb.HBError) as e:
            srv.submit(bad_off, idx, 4, 1)
        assert e.value.status == hb.HB_EINVAL
        # 2 n p bytes over the budget: 2 * 5000 * 256 > 1 MiB
        big = gg.empty(5000)
        with pytest.raises(hb.HBError) as e:
            srv.submit(*big, 8, 1)
        assert e.value.status == hb.HB_ENOMEM and "budget" in str(e.value)
        # within the budget but over the node pool (4096 rows, one block reserved)
        with pytest.raises(hb.HBError) as e:
            srv.submit(*gg.empty(4040), 4, 1)
        assert e.value.status == hb.HB_ENOMEM and "pool" in str(e.value)
        # over the arc pool
        many = gg.complete(40)
        with pytest.raises(hb.HBError) as e:
            srv.submit(*many, 4, 1)
        assert e.value.status == hb.HB_ENOMEM
        st = srv.stats()
        assert st["submitted"] == 0 and st["queued"] == 0


def test_queued_requests_cancel_and_report_once(hb):
    off, idx = gg.undirected_path(50)
    with hb.Server(start_paused=True) as srv:
        reqs = [srv.submit(off, idx, 4, s) for s in range(3)]
        assert [r.id for r in reqs] == [1, 2, 3]
        for r in reqs:
            info = srv.poll(r)
            assert info["state_name"] == "queued" and info["t_admit"] == -1.0
        st = srv.stats()
        assert st["submitted"] == 3 and st["queued"] == 3 and st["admitted"] == 0
        for r in reqs:
            srv.cancel(r)
        with pytest.raises(hb.HBError) as e:
            srv.cancel(reqs[0])                       # no longer queued
        assert e.value.status == hb.HB_ESTATE
        info = srv.wait(reqs[0], 5.0)
        assert info["state_name"] == "cancelled"
        with pytest.raises(hb.HBError) as e:          # a final state is reported once
            srv.poll(reqs[0])
        assert e.value.status == hb.HB_EINVAL
        assert srv.poll(reqs[1])["state_name"] == "cancelled"
        st = srv.stats()
        assert st["cancelled"] == 3 and st["queued"] == 0 and st["admitted"] == 0
        with pytest.raises(hb.HBError) as e:
            srv.wait(reqs[1], 0.1)
        assert e.value.status == hb.HB_EINVAL
    # stopping a paused server whose requests were all cancelled touches no device


def test_wait_times_out_on_a_queued_request(hb):
    off, idx = gg.undirected_path(8)
    with hb.Server(start_paused=True) as srv:
        r = srv.submit(off, idx, 4, 7)
        with pytest.raises(hb.HBError) as e:
            srv.wait(r, 0.05)
        assert e.value.status == hb.HB_ESTATE and "timed out" in str(e.value)
        srv.cancel(r)
        assert srv.wait(r)["state_name"] == "cancelled"
