import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


def pytest_terminal_summary(terminalreporter):
    """What the GPU parity checks left out, per test: knife-edge pixels
    (compared at the looser bar) and Gaussians excluded from the gradient
    check, next to the totals."""
    rows = getattr(sys.modules.get('_parity'), 'REPORT', None)
    if not rows:
        return
    tr = terminalreporter
    tr.section('parity exclusions')
    tr.write_line(f"{'test':72s} {'tile':>4s} {'flagged px':>14s} {'stopped px':>10s} "
                  f"{'clamped':>8s} {'excluded G':>14s} {'(clamp)':>7s}")
    for r in rows:
        tr.write_line(f"{r['test'][-72:]:72s} {r['tile']:4d} "
                      f"{r['flagged_px']:6d}/{r['pixels']:<7d} {r['stopped_px']:10d} "
                      f"{r['clamped_blends']:8d} {r['excluded']:6d}/{r['gaussians']:<7d} "
                      f"{r['clamp_excluded']:7d}")
