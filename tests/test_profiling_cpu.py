"""Host-side summaries of rocprofv3 output (no GPU): kernel-name shortening, the per-kernel
table, the chain-span summary and the counter-based traffic figure."""
import csv

import pytest

import rocprof_summary as P


def _write(path, header, rows):
    with open(path, 'w', newline='') as fh:
        w = csv.writer(fh)
        w.writerow(header)
        w.writerows(rows)


def test_short_names():
    assert P.short_name('void mprk::k_gm_orth<__half, float, 4, 8, 4>(mprk::Launch)') == 'gm_orth'
    assert P.short_name('_ZN4mprk10k_residualILi4ELi0EEEvNS_6LaunchE') == 'residual'
    assert P.short_name('__amd_rocclr_copyBuffer') == '__amd_rocclr_copyBuffer'


def test_chain_summary_spans_include_the_gaps(tmp_path):
    k = 'void mprk::k_fdm_contract<float, float, float, 1, 1, 64, 32>(mprk::FdmGeo)'
    other = 'void mprk::k_cg_rz<float, float, 4, 0>(mprk::Launch)'
    rows, t = [], 0
    for run in range(3):
        for i in range(6):  # 10 us kernels, 2 us apart
            rows.append((k, t, t + 10_000))
            t += 12_000
        rows.append((other, t, t + 5_000))
        t += 7_000
    rows.append((k, t, t + 10_000))  # a lone dispatch is not a run of six
    path = tmp_path / 'trace.csv'
    _write(path, ['Kernel_Name', 'Start_Timestamp', 'End_Timestamp'], rows)
    text = P.chain_summary(str(path), 'fdm_contract', 6)
    assert 'runs: 3' in text
    assert 'kernel duration per launch, mean: 10.00 us' in text
    assert f'mean: {(5 * 12 + 10) / 6:.2f} us' in text
    last = P.chain_summary(str(path), 'fdm_contract', 6, last=2)
    assert 'last 2 runs: kernel duration per launch 10.00 us' in last


def test_traffic_scales_by_the_calibration_copy(tmp_path):
    k = 'void mprk::k_gm_orth<__half, float, 4, 8, 4>(mprk::Launch)'
    cp = '__amd_rocclr_copyBuffer'
    f = tmp_path / 'f.csv'
    w = tmp_path / 'w.csv'
    hdr = ['Dispatch_Id', 'Kernel_Name', 'Counter_Name', 'Counter_Value']
    # the copy of 1024 MiB reads as half its size in FETCH_SIZE, as its size in WRITE_SIZE
    _write(f, hdr, [(1, cp, 'FETCH_SIZE', 512 * 1024), (2, k, 'FETCH_SIZE', 1000),
                    (3, k, 'FETCH_SIZE', 3000), (4, k, 'FETCH_SIZE', 1)])
    _write(w, hdr, [(1, cp, 'WRITE_SIZE', 1024 * 1024), (2, k, 'WRITE_SIZE', 400),
                    (4, k, 'WRITE_SIZE', 2)])
    t = P.traffic(str(f), str(w), 'gm_orth', 1024)
    assert t['fetch_factor'] == pytest.approx(2.0)
    assert t['working_dispatches'] == 2  # the near-empty dispatch is counted apart
    assert t['fetch_bytes_per_worked_launch'] == pytest.approx(2000 * 1024 * 2.0)
    assert t['write_bytes_per_worked_launch'] == pytest.approx(400 * 1024)


def test_traffic_table_lists_every_library_kernel(tmp_path):
    ko = 'void mprk::k_gm_orth<__half, float, 4, 8, 4>(mprk::Launch)'
    kr = 'void mprk::k_residual_zm<4>(mprk::ZLaunch)'
    cp = '__amd_rocclr_copyBuffer'
    f = tmp_path / 'f.csv'
    w = tmp_path / 'w.csv'
    hdr = ['Dispatch_Id', 'Kernel_Name', 'Counter_Name', 'Counter_Value']
    _write(f, hdr, [(1, cp, 'FETCH_SIZE', 512 * 1024), (2, ko, 'FETCH_SIZE', 1000),
                    (3, kr, 'FETCH_SIZE', 250)])
    _write(w, hdr, [(1, cp, 'WRITE_SIZE', 1024 * 1024), (2, ko, 'WRITE_SIZE', 100),
                    (3, kr, 'WRITE_SIZE', 500)])
    text = P.traffic_table(str(f), str(w), 1024, unknowns=1024, command_fetch='cf', command_write='cw')
    rows = {ln.split()[0]: ln.split() for ln in text.splitlines() if ln.startswith(('gm_orth', 'residual_zm'))}
    assert set(rows) == {'gm_orth', 'residual_zm'}
    # gm_orth: (1000 * 2 + 100) KiB per dispatch over 1024 unknowns
    assert float(rows['gm_orth'][-1]) == pytest.approx(2100 * 1024 / 1024, rel=1e-3)
    assert 'cf' in text and 'cw' in text


def test_traffic_counts_only_dispatches_after_the_marker(tmp_path):
    k = 'void mprk::k_gm_orth<__half, float, 4, 8, 4>(mprk::Launch)'
    fill = 'mprk::k_fill_pattern(long, double, double, double*)'
    cp = '__amd_rocclr_copyBuffer'
    f = tmp_path / 'f.csv'
    w = tmp_path / 'w.csv'
    hdr = ['Dispatch_Id', 'Kernel_Name', 'Counter_Name', 'Counter_Value']
    # trial launches (9000 KiB) before the autotuner's last fill, measured ones (1000) after it
    _write(f, hdr, [(1, cp, 'FETCH_SIZE', 512 * 1024), (2, k, 'FETCH_SIZE', 9000),
                    (3, fill, 'FETCH_SIZE', 1), (4, k, 'FETCH_SIZE', 1000),
                    (5, k, 'FETCH_SIZE', 1000)])
    _write(w, hdr, [(1, cp, 'WRITE_SIZE', 1024 * 1024), (2, k, 'WRITE_SIZE', 900),
                    (3, fill, 'WRITE_SIZE', 5), (4, k, 'WRITE_SIZE', 100), (5, k, 'WRITE_SIZE', 100)])
    t = P.traffic(str(f), str(w), 'gm_orth', 1024, after='fill_pattern')
    assert t['dispatches'] == 2
    assert t['fetch_bytes_per_worked_launch'] == pytest.approx(1000 * 1024 * 2.0)
    assert t['write_bytes_per_worked_launch'] == pytest.approx(100 * 1024)
    assert P.traffic(str(f), str(w), 'gm_orth', 1024)['dispatches'] == 3
