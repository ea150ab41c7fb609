"""bench.py on the CPU: it measures one GPU and says so when asked for more, and the arithmetic
that turns rocprofv3's L2 request counters into bytes (the traffic figures of the summaries)."""

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, cwd=ROOT, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in (r.stdout + r.stderr)


@pytest.mark.parametrize("n", [0, -1])
def test_bench_refuses_no_gpus(n):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", str(n)], capture_output=True,
                       text=True, cwd=ROOT, timeout=120)
    assert r.returncode != 0


def test_request_counters_to_bytes():
    """A 1 GiB copy issues 2^23 reads of 128 bytes and 2^24 writes of 64 bytes: 1 GiB each way.
    Mixed sizes add up by request size; requests of no listed size count 64 bytes; rocprofv3's
    FETCH_SIZE expression takes TCC_BUBBLE as the 128-byte reads (0 here gives half the bytes)."""
    sys.path.insert(0, ROOT)
    import bench

    gib = 1 << 30
    c = {"TCC_EA0_RDREQ_sum": 2.0 ** 23, "TCC_EA0_RDREQ_32B_sum": 0.0, "TCC_EA0_RDREQ_64B_sum": 0.0,
         "TCC_EA0_RDREQ_128B_sum": 2.0 ** 23, "TCC_EA0_WRREQ_sum": 2.0 ** 24, "TCC_EA0_WRREQ_64B_sum": 2.0 ** 24,
         "TCC_BUBBLE_sum": 0.0, "TCC_HIT_sum": 1.0, "TCC_MISS_sum": 3.0}
    b = bench._bytes_of(c)
    assert b["read_bytes"] == gib and b["write_bytes"] == gib
    assert b["fetch_size_expression_bytes"] == gib / 2
    assert b["l2_hit_rate"] == 0.25
    c = {"TCC_EA0_RDREQ_sum": 10.0, "TCC_EA0_RDREQ_32B_sum": 1.0, "TCC_EA0_RDREQ_64B_sum": 2.0,
         "TCC_EA0_RDREQ_128B_sum": 3.0, "TCC_EA0_WRREQ_sum": 5.0, "TCC_EA0_WRREQ_64B_sum": 2.0}
    b = bench._bytes_of(c)
    assert b["read_bytes"] == 32 * 1 + 64 * 2 + 128 * 3 + 64 * 4
    assert b["write_bytes"] == 32 * 3 + 64 * 2


def test_counter_summary_reads_rocprof_csv(tmp_path):
    """Per (kernel, workgroups): the mean per dispatch of each counter, and the bytes from it."""
    sys.path.insert(0, ROOT)
    import bench

    head = "Dispatch_Id,Kernel_Name,Grid_Size,Workgroup_Size,Counter_Name,Counter_Value\n"
    rows = ["1,\"void epk::reduce_kernel<5, false>(epk::DevPlan)\",1024,256,TCC_EA0_RDREQ_sum,100",
            "1,\"void epk::reduce_kernel<5, false>(epk::DevPlan)\",1024,256,TCC_EA0_RDREQ_128B_sum,100",
            "2,\"void epk::reduce_kernel<5, false>(epk::DevPlan)\",1024,256,TCC_EA0_RDREQ_sum,300",
            "2,\"void epk::reduce_kernel<5, false>(epk::DevPlan)\",1024,256,TCC_EA0_RDREQ_128B_sum,300"]
    path = tmp_path / "c.csv"
    path.write_text(head + "\n".join(rows) + "\n")
    t = bench._counter_table([str(path)])
    (key, d), = t.items()
    assert key[1] == 4 and d["TCC_EA0_RDREQ_sum"] == 200.0
    md = bench.summarize_counters([str(path)])
    assert "| 4 | 2 |" in md and "| 0.0 |" in md  # 200 requests of 128 bytes: 25,600 bytes = 0.0 MB
