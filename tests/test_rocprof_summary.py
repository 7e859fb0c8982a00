"""The profile summariser's choice of the calibration copy and its kernel
names, on hand-made rocprofv3 CSV rows."""
import csv

from paper_1303_0107_amd import rocprof_summary as R

FIELDS = ["Dispatch_Id", "Grid_Size", "Kernel_Name", "Counter_Name", "Counter_Value"]


def _write(path, rows):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, FIELDS)
        w.writeheader()
        for r in rows:
            w.writerow(dict(zip(FIELDS, r)))


def test_calibration_copy_is_found_by_its_write_reading(tmp_path):
    """A program whose largest copy is not the calibration copy: the copy whose
    write reading is the calibration size is taken, with the fetch reading of
    the same dispatch."""
    n = 1 << 28
    fetch = [(1, 131072, "__amd_rocclr_copyBuffer", "FETCH_SIZE", n / 2048),
             (2, 131072, "__amd_rocclr_copyBuffer", "FETCH_SIZE", 1.125 * n / 2048),
             (3, 4096, "k", "FETCH_SIZE", 10.0)]
    write = [(1, 131072, "__amd_rocclr_copyBuffer", "WRITE_SIZE", n / 1024),
             (2, 131072, "__amd_rocclr_copyBuffer", "WRITE_SIZE", 1.125 * n / 1024),
             (3, 4096, "k", "WRITE_SIZE", 5.0)]
    _write(tmp_path / "f.csv", fetch)
    _write(tmp_path / "w.csv", write)
    f, nf, cf = R.per_kernel(str(tmp_path / "f.csv"), "FETCH_SIZE")
    w, nw, cw = R.per_kernel(str(tmp_path / "w.csv"), "WRITE_SIZE")
    assert R.copy_readings(cf, cw, n) == (n / 2048, n / 1024)
    assert f[("k", 4096)] == 10.0 and nw[("k", 4096)] == 1
    # without an exact reading, the largest copy
    assert R.copy_readings([1.0, 3.0], [2.0, 6.0], n) == (3.0, 6.0)


def test_kernel_names_keep_anonymous_namespace_kernels():
    assert R.short("lbm::(anonymous namespace)::narrow_kernel<16>(lbm::(anonymous "
                   "namespace)::Cand const*)") == "narrow_kernel<16>"
    assert R.short("void lbm::sweep::tb_kernel<lbm::OffsetCell<float, float, float>, 32, 9>"
                   "(args)") == "tb_kernel<F32Cell, 32, 9>"


def test_mangled_half_precision_sweep_names():
    name = ("_ZN3lbm5sweep9tb_kernelINS_10OffsetCellIDF16_ffEELi32ELi9ELi1024ELi0ELb0ELb1EEEv"
            "NS_9SweepArgsINT_1TEEEPKii")
    assert R.short(name) == "tb_kernel<H16Cell, 32, 9, 1024, 0, false, true>"
