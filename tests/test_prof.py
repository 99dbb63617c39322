"""Host-side checks of the rocprofv3 summary tool that feeds the bench's
traffic figure: calibration by the copy dispatch and the per-launch sum."""
import csv
import hashlib

from paper_2007_08555_amd import prof

FIELDS = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]


def _write(path, counter, rows):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=FIELDS)
        w.writeheader()
        for d, (name, v) in enumerate(rows):
            w.writerow({"Dispatch_Id": d, "Kernel_Name": name, "Counter_Name": counter, "Counter_Value": v})


def test_traffic_is_calibrated_by_the_copy(tmp_path):
    # the copy of 1 MiB reads as 512 KiB fetched and 1024 KiB written: factors 2 and 1
    fetch = [("__amd_rocclr_copyBuffer", 1.0), ("__amd_rocclr_copyBuffer", 512.0),
             ("void lev16::moments_kernel(x)", 100.0), ("void lev16::adjoint(x)", 50.0),
             ("other_kernel", 999.0), ("void lev16::moments_kernel(x)", 100.0), ("void lev16::adjoint(x)", 70.0)]
    write = [("__amd_rocclr_copyBuffer", 2.0), ("__amd_rocclr_copyBuffer", 1024.0),
             ("void lev16::moments_kernel(x)", 10.0), ("void lev16::adjoint(x)", 20.0),
             ("other_kernel", 999.0), ("void lev16::moments_kernel(x)", 30.0), ("void lev16::adjoint(x)", 20.0)]
    _write(tmp_path / "f.csv", "FETCH_SIZE", fetch)
    _write(tmp_path / "w.csv", "WRITE_SIZE", write)
    src = tmp_path / "k.hip"
    # the hash covers the lines that the FP64 evaluation part compiles
    src.write_text("common\n#if MTP_PART == 3\nloss only\n#endif\n#if MTP_PART == 1 || MTP_PART == 2\neval\n#endif\n")
    out = tmp_path / "t.md"
    prof.traffic(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), str(out), "cmd f", "cmd w", "title", "1",
                 r"lev16::(moments|adjoint)", str(src))
    fields = dict(line.split(": ", 1) for line in out.read_text().splitlines() if ": " in line)
    # per launch: moments read 100*2, written 20 (mean); adjoint read 60*2, written 20 (KiB)
    expect = (200 + 20 + 120 + 20) * 1024
    assert abs(float(fields["traffic_bytes_per_launch"]) - expect) <= 1e-6 * expect
    assert fields["kernel_part_sha256"] == hashlib.sha256(b"common\neval\n").hexdigest()
