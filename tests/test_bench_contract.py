"""Host-side contract of bench.py: one GPU only, the measured-traffic record
it reads from the committed profile, and the per-GPU share of its design
study of several GPUs."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]


def test_profile_traffic_is_read_only_for_the_current_sources():
    sys.path.insert(0, ROOT)
    import bench
    path = os.path.join(ROOT, "profiles", "k_brick_fp32c_c3_4M_traffic.md")
    vals = dict(line.split(":", 1) for line in open(path)
                if ":" in line and not line.startswith(("#", "|", "`")))
    vals = {k.strip(): v.strip() for k, v in vals.items()}
    stored = float(vals["traffic_bytes_per_launch"])
    # a byte count per launch a little above the algorithmic 20 + 2 n_mean
    # bytes per atom-substep (n_mean = 20.41 on the 4M-atom system)
    assert 1.0 < stored / (4_000_000 * 60.8) < 1.3
    fresh = vals["csrc_sha256"] == bench.library_source_hash()
    assert bench.measured_traffic("k_brick_fp32c", 4_000_000) == (stored if fresh else None)
    assert bench.measured_traffic("k_brick_fp32c", 1_000_000) is None
    assert bench.measured_traffic("k_no_such_kernel", 4_000_000) is None


def test_c3_shard_partitions_the_system_with_ghost_layers():
    """The per-GPU share of the bench's design study: over N slabs every atom
    is owned exactly once, and each share's ghosts are the atoms of the other
    slabs within r_c of its faces (periodic in x), placed inside its free-x box."""
    sys.path.insert(0, ROOT)
    import numpy as np
    import workloads as W
    w = W.c3(n_cells=12, n_substeps=1)
    s = w.systems[0]
    Lx, rc = float(s.box_len[0]), float(w.r_cut)
    for n in (2, 3, 4):
        owned = 0
        for part in range(n):
            sh, ghost = W.c3_shard(w, n, part)
            assert sh.pos.shape[1] == ghost.size == sh.T_e0.size == sh.mass.size
            assert list(sh.periodic) == [0, 1, 1]
            x = sh.pos[0]
            assert np.all(x > sh.box_lo[0]) and np.all(x < sh.box_lo[0] + sh.box_len[0])
            width = Lx / n
            own = ghost == 0.0
            assert np.all((x[own] >= 0.0) & (x[own] < width))
            assert np.all(((x[~own] >= -rc) & (x[~own] < 0.0)) |
                          ((x[~own] >= width) & (x[~own] < width + rc)))
            # brute force: the ghosts are exactly the other slabs' atoms within r_c of a face
            d = np.mod(s.pos[0] - part * width, Lx)
            want = int(np.count_nonzero(((d >= width) & (d < width + rc)) | (d >= Lx - rc)))
            assert int(ghost.sum()) == want
            owned += int(own.sum())
        assert owned == s.n


def test_every_profile_names_a_command_of_the_committed_bench():
    """Each rocprofv3 summary under profiles/ gives the command that made it;
    every such command runs bench.py (a committed file) with options that
    bench.py still accepts."""
    import glob
    import shlex
    sys.path.insert(0, ROOT)
    import bench
    files = sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md")))
    assert files
    for path in files:
        cmds = [line.strip() for line in open(path) if line.strip().startswith("rocprofv3 ")]
        assert cmds, f"{os.path.basename(path)} names no rocprofv3 command"
        for cmd in cmds:
            argv = shlex.split(cmd)
            assert "--" in argv, cmd
            prog = argv[argv.index("--") + 1:]
            assert prog[:2] == ["python", "bench.py"], cmd
            bench.make_parser().parse_args(prog[2:])   # exits (SystemExit) on an unknown option
