"""Summaries of rocprofv3 output for the library's kernels (measurement tooling beside bench.py;
not part of the library).

Two inputs are understood:
- the `*_kernel_stats.csv` of a `rocprofv3 --kernel-trace --stats --output-format csv` run, turned
  into a short text table (calls, average and total duration, share) with the command that made it,
  optionally with the span of runs of back-to-back dispatches of one kernel from the trace;
- two `rocprofv3 --pmc FETCH_SIZE` / `--pmc WRITE_SIZE` runs of a command that starts with a plain
  device copy of known size (`bench.py --calib-copy MIB`), turned into the HBM bytes one dispatch of
  a kernel moves.  Each counter is scaled by what it reads for that copy: the copy reads MIB and
  writes MIB, so factor = MIB * 1024 / counter (both counters are in KiB).

Usage:
  python rocprof_summary.py stats STATS_CSV --command CMD --out FILE \
      [--trace TRACE_CSV --chain fdm_contract:6[:LAST]]
  python rocprof_summary.py traffic FETCH_CSV WRITE_CSV --kernel gm_orth \
      --workload advdiff256 --calib-mib 1024 --command-fetch CMD --command-write CMD --out FILE
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os

ROOT = os.path.dirname(os.path.abspath(__file__))


def kernel_source_hash() -> str:
    """Hash of every library source (kernel bodies, device helpers, the engine's and runtime's
    launch order and shapes); a traffic figure is valid only for the sources it was taken on."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, 'paper_2412_16638_amd', 'csrc')
    for f in sorted(os.listdir(csrc)):
        if f.endswith(('.hpp', '.hip')):
            with open(os.path.join(csrc, f), 'rb') as fh:
                h.update(f.encode())
                h.update(fh.read())
    return h.hexdigest()[:16]


def short_name(name: str) -> str:
    """`mprk::k_gm_orth<...>(...)` or its mangled form `_ZN4mprk9k_gm_orth...` -> `gm_orth`;
    names outside the library pass through."""
    ident = ''
    if name.startswith('_ZN4mprk'):
        rest = name[len('_ZN4mprk'):]
        k = 0
        while k < len(rest) and rest[k].isdigit():
            k += 1
        if k:
            ident = rest[k:k + int(rest[:k])]
    else:
        i = name.find('mprk::')
        if i >= 0:
            for c in name[i + len('mprk::'):]:
                if not (c.isalnum() or c == '_'):
                    break
                ident += c
    if ident.startswith('k_'):
        return ident[2:]
    return ident or name


def stats_summary(stats_csv: str, command: str, top: int = 14) -> str:
    """Per kernel (template variants of one kernel summed), then per variant."""
    rows = list(csv.DictReader(open(stats_csv)))
    total = sum(float(r['TotalDurationNs']) for r in rows)
    agg = {}
    for r in rows:
        k = short_name(r['Name'])
        a = agg.setdefault(k, [0, 0.0])
        a[0] += int(r['Calls'])
        a[1] += float(r['TotalDurationNs'])
    lines = ['# rocprofv3 kernel statistics', '', f'command: {command}', '',
             '## per kernel (all template variants)', '',
             f'{"kernel":<24} {"calls":>6} {"avg_us":>10} {"total_ms":>10} {"share":>7}']
    for k, (n, t) in sorted(agg.items(), key=lambda kv: -kv[1][1])[:top]:
        lines.append(f'{k:<24} {n:>6} {t / n / 1e3:>10.2f} {t / 1e6:>10.3f} {t / total:>7.2%}')
    lines += ['', '## per template variant', '',
              f'{"kernel":<24} {"calls":>6} {"avg_us":>10} {"total_ms":>10} {"share":>7}  template']
    for r in rows[:top]:
        nm = r['Name']
        lines.append(f'{short_name(nm):<24} {int(r["Calls"]):>6} '
                     f'{float(r["AverageNs"]) / 1e3:>10.2f} {float(r["TotalDurationNs"]) / 1e6:>10.3f} '
                     f'{float(r["TotalDurationNs"]) / total:>7.2%}  {nm[:110]}')
    return '\n'.join(lines) + '\n'


def _counter_rows(path: str, counter: str):
    out = []
    for r in csv.DictReader(open(path)):
        if r['Counter_Name'] == counter:
            out.append(r)
    return out


def _calibration(rows, mib: int) -> float:
    """Largest __amd_rocclr_copyBuffer dispatch is the calibration copy of `mib` MiB."""
    copies = [float(r['Counter_Value']) for r in rows if 'copyBuffer' in r['Kernel_Name']]
    if not copies:
        raise ValueError('no calibration copy in the counter file')
    return mib * 1024.0 / max(copies)


def _after(rows, kernel: str):
    """The rows dispatched after the last dispatch of `kernel` (all rows if it never ran)."""
    marks = [int(r['Dispatch_Id']) for r in rows if short_name(r['Kernel_Name']) == kernel]
    if not marks:
        return rows
    last = max(marks)
    return [r for r in rows if int(r['Dispatch_Id']) > last]


def traffic(fetch_csv: str, write_csv: str, kernel: str, calib_mib: int,
            worked_frac: float = 0.01, after: str = None) -> dict:
    """Mean HBM bytes per working dispatch of `kernel` (dispatches that fetched less than
    `worked_frac` of the largest one had nothing left to do and are counted apart).  after:
    count only dispatches after the last one of that kernel (the autotuner's fill kernel marks
    the end of its trial runs, whose Krylov cycles differ from the measured steps')."""
    fr = _counter_rows(fetch_csv, 'FETCH_SIZE')
    wr = _counter_rows(write_csv, 'WRITE_SIZE')
    ff, fw = _calibration(fr, calib_mib), _calibration(wr, calib_mib)
    if after:
        fr, wr = _after(fr, after), _after(wr, after)
    fmine = [float(r['Counter_Value']) for r in fr if short_name(r['Kernel_Name']) == kernel]
    wmine = [float(r['Counter_Value']) for r in wr if short_name(r['Kernel_Name']) == kernel]
    if not fmine or not wmine:
        raise ValueError(f'kernel {kernel} not found in the counter files')
    big = max(fmine)
    fw_ = [v for v in fmine if v >= worked_frac * big]
    wbig = max(wmine)
    ww_ = [v for v in wmine if v >= worked_frac * wbig]
    fetch_b = sum(fw_) / len(fw_) * 1024 * ff
    write_b = sum(ww_) / len(ww_) * 1024 * fw
    return {'kernel': kernel, 'fetch_factor': ff, 'write_factor': fw,
            'counted_after': after, 'dispatches': len(fmine), 'working_dispatches': len(fw_),
            'fetch_bytes_per_worked_launch': fetch_b, 'write_bytes_per_worked_launch': write_b,
            'bytes_per_worked_launch': fetch_b + write_b}


def traffic_table(fetch_csv: str, write_csv: str, calib_mib: int, unknowns: int,
                  command_fetch: str, command_write: str, after: str = None) -> str:
    """HBM bytes per working dispatch, and per unknown, of every library kernel in the two
    counter runs, as a text table (after: as in traffic)."""
    fr = _counter_rows(fetch_csv, 'FETCH_SIZE')
    sel = _after(fr, after) if after else fr
    names = sorted({short_name(r['Kernel_Name']) for r in sel
                    if 'mprk' in r['Kernel_Name'] and short_name(r['Kernel_Name']) != r['Kernel_Name']})
    ff = _calibration(fr, calib_mib)
    fw = _calibration(_counter_rows(write_csv, 'WRITE_SIZE'), calib_mib)
    lines = ['# HBM traffic per working dispatch (rocprofv3 FETCH_SIZE / WRITE_SIZE)', '',
             f'command (FETCH_SIZE): {command_fetch}', f'command (WRITE_SIZE): {command_write}',
             f'calibration: plain device copy of {calib_mib} MiB; fetch factor {ff:.4f}, '
             f'write factor {fw:.4f}', f'kernel sources: {kernel_source_hash()}',
             f'dispatches counted: ' + (f'after the last {after}' if after else 'all'), '',
             f'{"kernel":<22}{"dispatches":>11}{"working":>9}{"fetch MB":>11}{"write MB":>11}'
             f'{"B/unknown":>11}']
    for k in names:
        try:
            t = traffic(fetch_csv, write_csv, k, calib_mib, after=after)
        except ValueError:
            continue
        lines.append(f'{k:<22}{t["dispatches"]:>11}{t["working_dispatches"]:>9}'
                     f'{t["fetch_bytes_per_worked_launch"] / 1e6:>11.2f}'
                     f'{t["write_bytes_per_worked_launch"] / 1e6:>11.2f}'
                     f'{t["bytes_per_worked_launch"] / unknowns:>11.2f}')
    return '\n'.join(lines) + '\n'


def chain_summary(trace_csv: str, kernel: str, n: int, last: int = 0) -> str:
    """Runs of exactly n back-to-back dispatches of `kernel` (no other kernel between them, in
    dispatch order): the span from the first start to the last end, per launch.  This is what an
    event pair around the n launches measures (the kernels plus the gaps between them).  last > 0
    also reports the last `last` runs alone (the bench's profiled pass comes last)."""
    rows = sorted(csv.DictReader(open(trace_csv)), key=lambda r: int(r['Start_Timestamp']))
    spans, durs, run = [], [], []
    for r in rows + [None]:
        if r is not None and short_name(r['Kernel_Name']) == kernel:
            run.append(r)
            continue
        if len(run) == n:
            t0 = int(run[0]['Start_Timestamp'])
            t1 = int(run[-1]['End_Timestamp'])
            spans.append((t1 - t0) / n)
            durs += [int(x['End_Timestamp']) - int(x['Start_Timestamp']) for x in run]
        run = []
    if not spans:
        return f'\n## {kernel}: no runs of {n} back-to-back dispatches\n'
    text = (f'\n## {kernel}: runs of {n} back-to-back dispatches (one event pair in the bench)\n\n'
            f'runs: {len(spans)}\n'
            f'kernel duration per launch, mean: {sum(durs) / len(durs) / 1e3:.2f} us\n'
            f'span per launch (first start to last end / {n}), mean: '
            f'{sum(spans) / len(spans) / 1e3:.2f} us\n')
    if 0 < last <= len(spans):
        tail_d = durs[-last * n:]
        text += (f'last {last} runs: kernel duration per launch {sum(tail_d) / len(tail_d) / 1e3:.2f} us, '
                 f'span per launch {sum(spans[-last:]) / last / 1e3:.2f} us\n')
    return text


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest='what', required=True)
    a = sub.add_parser('stats')
    a.add_argument('csv')
    a.add_argument('--command', required=True)
    a.add_argument('--out', required=True)
    a.add_argument('--trace', help='kernel trace csv, for --chain')
    a.add_argument('--chain', help='KERNEL:N[:LAST], summarise runs of N back-to-back dispatches '
                                   '(and the last LAST of them alone)')
    b = sub.add_parser('traffic')
    b.add_argument('fetch_csv')
    b.add_argument('write_csv')
    b.add_argument('--kernel', required=True)
    b.add_argument('--workload', required=True)
    b.add_argument('--calib-mib', type=int, required=True)
    b.add_argument('--command-fetch', required=True)
    b.add_argument('--command-write', required=True)
    b.add_argument('--out', required=True)
    b.add_argument('--after-kernel', help='count only dispatches after the last one of this kernel')
    t = sub.add_parser('traffic-table')
    t.add_argument('fetch_csv')
    t.add_argument('write_csv')
    t.add_argument('--calib-mib', type=int, required=True)
    t.add_argument('--unknowns', type=int, required=True)
    t.add_argument('--command-fetch', required=True)
    t.add_argument('--command-write', required=True)
    t.add_argument('--out', required=True)
    t.add_argument('--after-kernel', help='count only dispatches after the last one of this kernel')
    args = ap.parse_args()
    if args.what == 'traffic-table':
        with open(args.out, 'w') as fh:
            fh.write(traffic_table(args.fetch_csv, args.write_csv, args.calib_mib, args.unknowns,
                                   args.command_fetch, args.command_write, args.after_kernel))
        return
    if args.what == 'stats':
        text = stats_summary(args.csv, args.command)
        if args.chain:
            parts = args.chain.split(':')
            text += chain_summary(args.trace, parts[0], int(parts[1]),
                                  int(parts[2]) if len(parts) > 2 else 0)
        with open(args.out, 'w') as fh:
            fh.write(text)
    else:
        t = traffic(args.fetch_csv, args.write_csv, args.kernel, args.calib_mib,
                    after=args.after_kernel)
        t.update({'workload': args.workload, 'kernel_hash': kernel_source_hash(),
                  'command_fetch': args.command_fetch, 'command_write': args.command_write,
                  'calibration': f'plain device copy of {args.calib_mib} MiB (reads and writes '
                                 f'{args.calib_mib} MiB)'})
        with open(args.out, 'w') as fh:
            json.dump(t, fh, indent=1)
            fh.write('\n')


if __name__ == '__main__':
    main()
