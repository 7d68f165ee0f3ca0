"""The oracle's C sources under AddressSanitizer and UndefinedBehaviorSanitizer.

oracle/sanitize_main.c drives every oracle routine (assembly on real and
complex states, both hierarchies under several parameter sets, the V-cycle,
the block preconditioner variants, GMRES with and without restarts, ILU(0)
and CPR, the network's features, forward pass and gradient) on small grids:
3-D, a 2-D slab with the Bennison viscosity and a diagonal permeability
tensor, and a single row of cells.  Built with gcc (host code only) and run
as its own process; any invalid access, leak or undefined operation fails
it."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = ["physics.c", "amg.c", "krylov.c", "cnn.c", "ilu.c", "sanitize_main.c"]


def test_oracle_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_sanitize")
    odir = os.path.join(ROOT, "oracle")
    cmd = ["gcc", "-std=gnu99", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-Wall", "-Wno-unused-function",
           "-Wno-maybe-uninitialized", "-o", exe] + [os.path.join(odir, s) for s in SRC] + ["-lm"]
    subprocess.run(cmd, check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    assert r.stdout.startswith("sanitize ok"), r.stdout
