"""Host logic of bench.py on the CPU: the source hash that keys the traffic table, the traffic
table and the pipeline counter table built from rocprofv3 files, and the bytes model."""
import csv
import os

import bench


def test_code_text_ignores_comments_and_layout():
    a = 'int f(int x) {\n  return x + 1;  // add one\n}\n/* block\n comment */ const char* s = "a // b";\n'
    b = ('int f(int x)\n{ return x + 1; }\n// another comment\nconst char* s = '
         '"a // b"; /* tail */\n')
    assert bench.code_text(a).replace(" ", "") == bench.code_text(b).replace(" ", "")
    assert '"a // b"' in bench.code_text(a)           # a literal keeps its slashes
    assert "add one" not in bench.code_text(a)
    assert bench.code_text("x = 1;") != bench.code_text("x = 2;")


def _write(path, header, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(header)
        w.writerows(rows)


def _counters(path, dispatches):
    hdr = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]
    rows = []
    for d, (name, vals) in enumerate(dispatches):
        for c, v in vals.items():
            rows.append([d, name, c, v])
    _write(path, hdr, rows)


def test_traffic_table_from_counters(tmp_path):
    d = str(tmp_path)
    _write(os.path.join(d, "trace", "rmat24_kernel_stats.csv"),
           ["Name", "Calls", "AverageNs", "MinNs", "MaxNs", "Percentage"],
           [["void k_spmv_csbr<double, double, 4, true>(int const*)", 2, 800000, 790000, 810000,
             90.0]])
    gib2 = 2 << 30
    copy = "__amd_rocclr_copyBuffer"
    kern = "void k_spmv_csbr<double, double, 4, true>(int const*)"
    # the copy's counters read twice its 2 GiB: every kernel's bytes are halved
    _counters(os.path.join(d, "fetch", "rmat24_counter_collection.csv"), [
        (copy, {"TCC_EA0_RDREQ_32B": 0, "TCC_EA0_RDREQ_64B": 0,
                "TCC_EA0_RDREQ_128B": 2 * gib2 // 128, "TCC_EA0_RDREQ": 2 * gib2 // 128}),
        (kern, {"TCC_EA0_RDREQ_32B": 4, "TCC_EA0_RDREQ_64B": 10, "TCC_EA0_RDREQ_128B": 1000,
                "TCC_EA0_RDREQ": 1014}),
        (kern, {"TCC_EA0_RDREQ_32B": 0, "TCC_EA0_RDREQ_64B": 0, "TCC_EA0_RDREQ_128B": 3000,
                "TCC_EA0_RDREQ": 3000})])
    _counters(os.path.join(d, "write", "rmat24_counter_collection.csv"), [
        (copy, {"TCC_EA0_WRREQ": gib2 // 64, "TCC_EA0_WRREQ_64B": gib2 // 64}),
        (kern, {"TCC_EA0_WRREQ": 30, "TCC_EA0_WRREQ_64B": 10}),
        (kern, {"TCC_EA0_WRREQ": 0, "TCC_EA0_WRREQ_64B": 0})])
    md, tj = bench.summarize_rocprof(d, "rmat24")
    reads = ((32 * 4 + 64 * 10 + 128 * 1000) + 128 * 3000) / 2 * 0.5   # mean x calibration 1/2
    writes = (32 * (30 - 10) + 64 * 10) / 2 * 1.0                      # write calibration 1
    got = tj["traffic_bytes_per_launch"]["k_spmv_csbr"]
    assert abs(got - (reads + writes)) < 1e-6, (got, reads + writes)
    assert "bytes read x 0.5000, bytes written x 1.0000" in md
    assert tj["kernel_src"] == bench.src_hash(*bench.KERNEL_SOURCES)


def test_pipeline_table(tmp_path):
    d = str(tmp_path)
    kern = "void k_spmv_csbr<double, double, 4, true>(int const*)"
    one = {"GRBM_GUI_ACTIVE": 8 * 1000, "TA_TA_BUSY_sum": 256 * 800, "TD_TD_BUSY_sum": 256 * 900,
           "SQ_INSTS_VALU": 2e6, "SQ_INSTS_LDS": 3e6, "SQ_INSTS_VMEM_RD": 4e6}
    _counters(os.path.join(d, "rmat24_counter_collection.csv"),
              [(kern, one), (kern, one), ("void k_other(int)", one)])
    md = bench.summarize_pipe(d, "rmat24")
    assert "| `k_spmv_csbr` | 2 | 80% | 90% | 2.0 | 3.0 | 4.0 |" in md
    assert "k_other" not in md


class _Parts:
    def __init__(self, parts):
        self.parts = parts


def test_bytes_model_crs():
    m, nnz, nt = 1000, 50_000, 900
    base = 12 * nnz + 8 * (nt + m) + 4 * (m + 1)
    assert bench.spmv_bytes("rowsplit", m, nnz, nt, _Parts(7)) == base + 4 * 8
    assert bench.spmv_bytes("merge", m, nnz, nt, _Parts(7)) == base + 8 * 8 + 12 * 7
    # reduced precision: 4 + value bytes per entry, FP32 vectors
    assert bench.spmv_bytes("rowsplit", m, nnz, nt, _Parts(7), val_bytes=2, vec_bytes=4) == \
        6 * nnz + 4 * (nt + m) + 4 * (m + 1) + 4 * 8
