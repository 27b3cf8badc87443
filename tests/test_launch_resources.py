"""Launch resources of every compiled operator and face kernel, from the compiler's own
report (hipcc -Rpass-analysis=kernel-resource-usage, which the build keeps beside each
object file) and the block sizes of the LDS plan (tests/emul/plan_check.cpp).

The launch plan picks block sizes so that registers, not LDS, set the occupancy: a
128-thread workgroup relies on four of them fitting in a compute unit's 160 KB of LDS
for two waves per SIMD, LDS counted in whole 1280-byte granules (128 per compute unit).  The plan sizes LDS from its own arithmetic plus an allowance
for the small per-workgroup variables; these tests check the compiler's actual
figures: every kernel exists for every supported (degree, n_q) in both precisions and
both metric forms, LDS allows at least as many waves per SIMD as the registers do (up
to the two the register budget aims at), and the float32 kernels and the float64
kernels of degree <= 3 do not spill.  The streamed kernels of degrees 8..15: every one
is reported, none spills (except the float64 face kernels at k = 14, 15, held to two waves
per SIMD, within the 32 dwords their plan was measured with), the cell kernel's LDS plan
leaves at least two workgroups per compute unit, and the float64 face kernels that keep
their traces inside the sweep area reach the workgroups per compute unit they are planned
for (four 128-thread workgroups at k = 8..10, n_q = k+1; two of 256 threads at k = 13..15).  Runs on the CPU; builds the library if no resource report is present.
"""
import glob
import os
import re
import subprocess
import tempfile

import pytest

from tests import emul_driver as ed

BUILD = os.path.join(ed.ROOT, "paper_1806_03095_amd", "_build")
LDS_GRANULE, LDS_GRANULES = 1280, 128   # a compute unit's 160 KB, allocated in granules
VGPR_FILE = 512          # VGPRs per lane of one SIMD's register file (wave64)


def _wg_per_cu(lds):
    return LDS_GRANULES // max(1, (lds + LDS_GRANULE - 1) // LDS_GRANULE)


def _reports(pattern="op_k*.resources.txt", count=7):
    files = sorted(glob.glob(os.path.join(BUILD, pattern)))
    if len(files) < count:
        from paper_1806_03095_amd import build as b
        b.build()
        files = sorted(glob.glob(os.path.join(BUILD, pattern)))
    out = {}
    for f in files:
        cur = None
        for line in open(f):
            m = re.search(r"Function Name: (\S+)", line)
            if m:
                cur = m.group(1)
                out[cur] = {}
                continue
            m = re.search(r"remark:\s+([A-Za-z ]+?)(?: \[[^\]]*\])?: (\S+) \[-Rpass", line)
            if m and cur:
                out[cur][m.group(1).strip()] = m.group(2)
    return out


def _block_sizes():
    with tempfile.TemporaryDirectory() as td:
        exe = os.path.join(td, "plan_check")
        cmd = ["g++", "-std=c++17", "-O0", "-Wno-unknown-pragmas", "-I", ed.EMU, "-I",
               os.path.join(ed.ROOT, "include"), "-I", ed.CSRC, os.path.join(ed.EMU, "plan_check.cpp"), "-o", exe]
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-4000:]
        out = subprocess.run([exe], capture_output=True, text=True).stdout
    blocks = {}
    for line in out.splitlines():
        m = re.match(r"k=(\d+) n_q=(\d+) (fp\d+): (face kernel )?.*?B=(\d+)", line)
        if m:
            blocks[(int(m.group(1)), int(m.group(2)), m.group(3), "face" if m.group(4) else "op")] = int(m.group(5))
    return blocks


def _supported(name="kSupported"):
    src = open(os.path.join(ed.CSRC, "dg_kernels.h")).read()
    start = re.search(name + r"\s*\[", src).start()
    body = src[start:src.index(";", start)]
    return [(int(a), int(b)) for a, b in re.findall(r"\{(\d+), (\d+)\}", body)]


@pytest.fixture(scope="module")
def table():
    rep, blocks = _reports(), _block_sizes()
    rows = {}
    for name, v in rep.items():
        m = re.match(r"_ZN4dgns\d+(dg_operator_kernel|dg_face_kernel)ILi(\d+)ELi(\d+)E([fd])Lb([01])E", name)
        if not m:
            continue
        kind = "op" if m.group(1) == "dg_operator_kernel" else "face"
        k, q = int(m.group(2)) - 1, int(m.group(3))
        prec = "fp64" if m.group(4) == "d" else "fp32"
        b = blocks[(k, q, prec, kind)]
        vg = int(v["VGPRs"]) + int(v["AGPRs"])
        lds = int(v["LDS Size"])
        rows[(k, q, prec, int(m.group(5)), kind)] = {
            "B": b, "vgpr": vg, "spill": int(v["VGPRs Spill"]), "scratch": int(v["ScratchSize"]), "lds": lds,
            "waves_vgpr": min(8, VGPR_FILE // ((vg + 7) // 8 * 8)),
            "waves_lds": _wg_per_cu(lds) * (b // 64) / 4.0}
    return rows


def test_every_supported_kernel_reported(table):
    for k, q in _supported():
        for prec in ("fp64", "fp32"):
            for gen in (0, 1):
                assert (k, q, prec, gen, "op") in table, (k, q, prec, gen)


def test_lds_does_not_lower_occupancy(table):
    bad = []
    for key, r in sorted(table.items()):
        want = min(2, r["waves_vgpr"])
        if r["waves_lds"] < want:
            bad.append((key, r))
    assert not bad, "\n".join("%s: %s" % b for b in bad)


def test_no_spills_where_the_budget_allows(table):
    bad = [(key, r) for key, r in sorted(table.items())
           if (key[2] == "fp32" or key[0] <= 3) and (r["spill"] or r["scratch"])]
    assert not bad, "\n".join("%s: %s" % b for b in bad)


def test_streamed_kernels_reported_spill_free_two_workgroups():
    rep = _reports("op_hd*.resources.txt", 3)
    def find(pat):
        hits = [v for n, v in rep.items() if re.match(pat, n)]
        assert len(hits) == 1, pat
        return hits[0]
    bad = []
    for k, q in _supported("kSupportedHd"):
        n = k + 1
        for t in ("d", "f"):
            for gen in (0, 1):
                cell = find(r"_ZN4dgns17dg_cell_hd_kernelILi%dELi%dE%sLb%dE" % (n, q, t, gen))
                face = find(r"_ZN4dgns17dg_face_hd_kernelILi%dELi%dE%sLb%dE" % (n, q, t, gen))
                minv = find(r"_ZN4dgns22inverse_mass_hd_kernelILi%dE%sLb%dE" % (n, t, gen))
                for what, v in (("cell", cell), ("face", face), ("minv", minv)):
                    allowed = 32 if (what == "face" and t == "d" and k >= 14) else 0
                    if int(v["VGPRs Spill"]) > allowed or (not allowed and int(v["ScratchSize"])):
                        bad.append((k, q, t, gen, what, v))
                if _wg_per_cu(int(cell["LDS Size"])) < 2:
                    bad.append((k, q, t, gen, "cell LDS", cell))
                if t == "d" and (q == n or k >= 13) and (q * q <= 128 or k >= 13):
                    # in-place traces: LDS and registers both allow the planned workgroups
                    threads = 128 if q * q <= 128 else 256
                    want = 4 if threads == 128 else 2
                    regs = int(face["VGPRs"]) + int(face["AGPRs"])
                    by_regs = (VGPR_FILE // max(1, (regs + 7) // 8 * 8)) * 4 // (threads // 64)
                    if min(_wg_per_cu(int(face["LDS Size"])), by_regs) < want:
                        bad.append((k, q, t, gen, "face workgroups", face))
    assert not bad, "\n".join("%s" % (b,) for b in bad)
