"""The host tile builder under AddressSanitizer and UBSan, without a GPU.

tests/host_builder/builder_check.cpp compiles paper_1609_01689_amd/csrc/build.cpp
(and the block-64 eigensolver) with g++ against a host stand-in of the HIP
runtime, builds the tile streams of a matrix (whole or in uneven slabs), checks
the invariants the SpMM kernel relies on (piece sizes and alignment, codes
inside their tile, the column order a permutation of the row order, the panel
order a permutation) and replays the kernel's two passes over the streams on
the CPU against the product computed from the CSR, within the componentwise
bound gamma_k |H||X| of the arithmetic precision.  The inputs cover the edge
cases of the format: n = 1, diagonal-only, empty rows, rows without a
diagonal entry, a trailing empty stretch, tiles cut into several pieces, both
code widths and both storage precisions."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HB = os.path.join(ROOT, "tests", "host_builder")
CSRC = os.path.join(ROOT, "paper_1609_01689_amd", "csrc")


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    if not shutil.which("g++") or not shutil.which("gcc"):
        pytest.skip("needs gcc/g++")
    d = tmp_path_factory.mktemp("hb")
    san = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-fno-sanitize-recover=undefined"]
    gen = str(d / "hsymgen.o")
    subprocess.run(["gcc", "-O1", "-g"] + san + ["-c", os.path.join(ROOT, "hsymgen", "hsymgen.c"), "-o", gen],
                   check=True)
    exe = str(d / "builder_check")
    cmd = (["g++", "-std=c++17", "-O1", "-g"] + san + ["-I" + HB, "-I" + CSRC,
           os.path.join(HB, "builder_check.cpp"), os.path.join(CSRC, "build.cpp"),
           os.path.join(CSRC, "symeig_host.cpp"), gen, "-lpthread", "-lm", "-o", exe])
    subprocess.run(cmd, check=True)
    return exe


CASES = [
    # case, n, N, seed, storage (0 fp64, 1 fp32), m, slab, r64, lc
    ("gen", 2000, 40, 1, 0, 8, 0, 0, 0),
    ("gen", 2000, 40, 1, 0, 16, 0, 0, 0),
    ("gen", 2000, 40, 1, 1, 16, 0, 0, 0),
    ("gen", 20000, 60, 7, 0, 16, 333, 0, 0),       # streaming create in uneven slabs
    ("gen", 20000, 60, 7, 1, 8, 1000, 0, 0),
    ("gen", 30000, 200, 3, 0, 16, 0, 7, 6),        # explicit R = 448, C = 64
    ("gen", 5000, 40, 9, 0, 1, 0, 0, 0),
    ("diag", 1, 0, 3, 0, 1, 0, 0, 0),
    ("diag", 300, 0, 1, 0, 16, 0, 0, 0),
    ("holes", 1, 0, 3, 0, 16, 0, 0, 0),
    ("holes", 300, 0, 3, 0, 16, 0, 0, 0),
    ("holes", 5000, 0, 4, 0, 4, 701, 0, 0),
    ("holes", 3000, 0, 5, 1, 4, 0, 16, 7),         # 32-bit codes (R * C = 2^17)
    ("dense", 900, 0, 5, 0, 16, 0, 7, 6),          # tiles cut into several pieces
    ("dense", 900, 0, 5, 1, 16, 0, 7, 6),
    ("dense", 700, 0, 5, 0, 1, 0, 4, 6),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: "-".join(str(x) for x in c))
def test_builder_under_sanitizers(checker, case):
    env = dict(os.environ, HSYM_HOST_THREADS="4", ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([checker] + [str(x) for x in case], capture_output=True, text=True, env=env, timeout=600)
    print(r.stdout)
    print(r.stderr[-4000:])
    assert r.returncode == 0 and r.stdout.strip().endswith("OK"), r.stdout + r.stderr[-4000:]


@pytest.mark.parametrize("N,rows", [(150, 512), (500, 384)])
def test_geometry_follows_tile_fill(checker, N, rows):
    """Without an explicit geometry the builder chooses the panels from the
    first rows it receives (fp32 storage, m = 16, n = 140,000: the default
    rule's 512 x 128 panels or 384 x 128 ones whose pieces hold 8,184 entries
    instead of 5,112).  At 150 nonzeros per full row the tiles of 512 rows
    fit one piece and the taller panels stay; at 500 they would be cut into
    about 1.6 pieces and the shorter panels are taken.  The
    replay of the kernel's passes checks the product either way."""
    env = dict(os.environ, HSYM_HOST_THREADS="4", ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([checker, "gen", "140000", str(N), "4", "1", "16", "0", "0", "0"], capture_output=True,
                       text=True, env=env, timeout=600)
    print(r.stdout)
    assert r.returncode == 0 and r.stdout.strip().endswith("OK"), r.stdout + r.stderr[-4000:]
    assert ("geometry R=%d C=128 " % rows) in r.stdout
