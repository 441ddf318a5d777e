"""Checks on the gfx950 machine code of the built sweep kernels (our own build,
disassembled with the ROCm LLVM tools; no GPU needed).

1. The SGPR-operand kernels issue groups of scalar loads from inline assembly.  A
scalar load writes its destination SGPRs some time after it issues, so a later
load of the same group must not take its address from registers that an
earlier, still outstanding load of the group writes: its address could change
under it.  The compiler never emits that for its own loads; this test makes sure
the register constraints of the hand-written groups rule it out as well.

2. The MFMA kernels read accumulator tiles from inline assembly (v_sad_u32).  The
compiler inserts the wait states between an MFMA and an ordinary VALU read of its
result, but not before an asm read, so the kernels add them by hand; the test
counts the wait states between every MFMA and the next instruction that reads its
destination registers.

3. The d-ary SGPR-operand kernels are compiled for a number of waves per SIMD
chosen per width; the Gray loop (the innermost loop that scores subsets) must
not spill at that register budget."""
import concurrent.futures
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BUILD = os.path.join(ROOT, "paper_2503_21596_amd", "_build")
LLVM = "/opt/rocm/llvm/bin"
TARGET = "hipv4-amdgcn-amd-amdhsa--gfx950"

LOAD = re.compile(r"\s+s_load_dword\w*\s+s\[(\d+):(\d+)\],\s+s\[(\d+):(\d+)\]")
LOAD1 = re.compile(r"\s+s_load_dword\s+s(\d+),\s+s\[(\d+):(\d+)\]")
FUNC = re.compile(r"^[0-9a-f]+ <(\S+)>:")


def _disassemble(obj, tmp_path):
    fat = tmp_path / (os.path.basename(obj) + ".fatbin")
    dev = tmp_path / (os.path.basename(obj) + ".gfx950.elf")
    subprocess.run([f"{LLVM}/llvm-objcopy", f"--dump-section=.hip_fatbin={fat}", obj], check=True)
    subprocess.run([f"{LLVM}/clang-offload-bundler", "--unbundle", "--type=o", f"--input={fat}",
                    f"--targets={TARGET}", f"--output={dev}"], check=True)
    r = subprocess.run([f"{LLVM}/llvm-objdump", "-d", "--mcpu=gfx950", str(dev)], check=True,
                       capture_output=True, text=True)
    return r.stdout.splitlines()


def scan(lines):
    """Scalar loads that read an address register written by an earlier scalar
    load with no s_waitcnt in between.  Returns (function, line) pairs."""
    bad = []
    fn = None
    pending = []          # destination ranges of loads issued since the last wait
    for line in lines:
        f = FUNC.match(line)
        if f:
            fn, pending = f.group(1), []
            continue
        if "s_waitcnt" in line or "s_endpgm" in line or "s_branch" in line or "s_cbranch" in line:
            pending = []
            continue
        m = LOAD.match(line)
        if m:
            d0, d1, b0, b1 = map(int, m.groups())
        else:
            m1 = LOAD1.match(line)
            if not m1:
                continue
            d0 = d1 = int(m1.group(1))
            b0, b1 = int(m1.group(2)), int(m1.group(3))
        if any(not (b1 < w0 or b0 > w1) for w0, w1 in pending):
            bad.append((fn, line.strip()))
        pending.append((d0, d1))
    return bad


MFMA = re.compile(r"\s+v_mfma\w*\s+v\[(\d+):(\d+)\]")
VRANGE = re.compile(r"v\[(\d+):(\d+)\]")
VONE = re.compile(r"(?<![\w\[:])v(\d+)")
MFMA_READ_WAITS = 24   # at least the longest XDL write -> VALU read requirement


def _vregs(text):
    out = set()
    for a, b in VRANGE.findall(text):
        out |= set(range(int(a), int(b) + 1))
    out |= {int(a) for a in VONE.findall(text)}
    return out


def mfma_short_reads(lines, need=MFMA_READ_WAITS):
    """Instructions that read a VGPR written by an MFMA fewer than `need` wait
    states after it (s_nop N counts N + 1, any other instruction 1), scanning each
    function in program order.  Returns (function, waits, line) triples."""
    bad = []
    fn = None
    pending = []   # [destination registers, wait states since the MFMA]
    for line in lines:
        f = FUNC.match(line)
        if f:
            fn, pending = f.group(1), []
            continue
        s = line.split("//")[0].split(";")[0].strip()
        if not s or s.endswith(":") or s.startswith("."):
            continue
        op = s.split()[0]
        operands = s[len(op):]
        srcs = _vregs(operands.split(",", 1)[1]) if "," in operands else set()
        for p in pending:
            if p[0] & srcs and p[1] < need:
                bad.append((fn, p[1], s))
        pending = [p for p in pending if not (p[0] & srcs)]
        w = int(s.split()[1], 0) + 1 if op == "s_nop" else 1
        for p in pending:
            p[1] += w
        m = MFMA.match(" " + s)
        if m:
            pending.append([set(range(int(m.group(1)), int(m.group(2)) + 1)), 0])
    return bad


def test_mfma_scan_catches_a_short_read():
    lines = ["0000000000000000 <k>:",
             "\tv_mfma_i32_32x32x16_i8 v[0:15], v[16:17], v[18:19], v[0:15]",
             "\ts_nop 7",
             "\tv_sad_u32 v20, v3, s4, v20"]
    assert len(mfma_short_reads(lines)) == 1
    ok = lines[:3] + ["\ts_nop 7", "\ts_nop 7", "\tv_sad_u32 v20, v21, s4, v20", lines[3]]
    assert mfma_short_reads(ok) == []


def test_scan_catches_a_redirected_load():
    """The scan flags the sequence the early-clobber constraints prevent."""
    lines = ["0000000000000000 <k>:",
             "\ts_load_dwordx8 s[36:43], s[36:37], 0x0",
             "\ts_load_dwordx8 s[44:51], s[36:37], 0x20",
             "\ts_waitcnt lgkmcnt(0)"]
    assert len(scan(lines)) == 1
    ok = ["0000000000000000 <k>:",
          "\ts_load_dwordx8 s[36:43], s[52:53], 0x0",
          "\ts_load_dwordx8 s[44:51], s[52:53], 0x20",
          "\ts_waitcnt lgkmcnt(0)",
          "\ts_load_dwordx2 s[52:53], s[52:53], 0x0"]
    assert scan(ok) == []


@pytest.mark.parametrize("obj", ["kbin0.o", "kbin1.o", "kbin2.o", "kdary.o", "kdarys0.o", "kdarys1.o", "kdarys2.o", "kdarys3.o", "kmfma0.o", "kmfma1.o", "kmfma2.o"])
def test_scalar_loads_keep_their_address(obj, tmp_path):
    path = os.path.join(BUILD, obj)
    if not os.path.exists(path):
        pytest.skip("library not built (run __graft_entry__.build())")
    if not os.path.exists(f"{LLVM}/llvm-objdump"):
        pytest.skip("ROCm LLVM tools not found")
    lines = _disassemble(path, tmp_path)
    assert sum(1 for l in lines if "s_load_dword" in l) > 100
    bad = scan(lines)
    assert not bad, bad[:5]


@pytest.mark.parametrize("obj", ["kmfma0.o", "kmfma1.o", "kmfma2.o"])
def test_mfma_results_wait(obj, tmp_path):
    path = os.path.join(BUILD, obj)
    if not os.path.exists(path):
        pytest.skip("library not built (run __graft_entry__.build())")
    if not os.path.exists(f"{LLVM}/llvm-objdump"):
        pytest.skip("ROCm LLVM tools not found")
    lines = _disassemble(path, tmp_path)
    assert sum(1 for l in lines if "v_mfma" in l) >= 32
    bad = mfma_short_reads(lines)
    assert not bad, bad[:5]


DEPTH = re.compile(r"^\s*;.*Depth=(\d+)")
DARY_S = re.compile(r"^(_ZN2ld9k_dary(32|16)sILi(\d+)ELi(\d+)E(?:Li(\d+)E)?EEvNS_5QArgsE):")


def gray_loop_spills(asm_lines):
    """Per k_dary32s / k_dary16s instantiation of a compiler assembly listing,
    keyed (bits, width, d, low rows; 0 where the name carries none): scratch
    instructions at the deepest loop level that holds v_sad_u32 or v_sad_u16 (the
    Gray loop)."""
    out = {}
    cur = None
    depth = 0
    for line in asm_lines:
        m = DARY_S.match(line)
        if m:
            cur = (int(m.group(2)), int(m.group(3)), int(m.group(4)), int(m.group(5) or 0))
            out[cur] = {"sad": {}, "scratch": {}}
            depth = 0
            continue
        if cur is None:
            continue
        if line.startswith(".Lfunc_end"):
            cur = None
            continue
        if re.match(r"^\.LBB\d+_\d+:", line):
            depth = 0
            continue
        d = DEPTH.match(line)
        if d:
            depth = int(d.group(1))
            continue
        if "v_sad_u32" in line or "v_sad_u16" in line:
            out[cur]["sad"][depth] = out[cur]["sad"].get(depth, 0) + 1
        if "scratch_" in line:
            out[cur]["scratch"][depth] = out[cur]["scratch"].get(depth, 0) + 1
    return {k: v["scratch"].get(max(v["sad"]), 0) for k, v in out.items() if v["sad"]}


def test_dary_gray_loop_has_no_spills(tmp_path):
    """Compiles the d-ary SGPR-operand kernels as the build does (same flags, full
    device pipeline) and keeps the compiler's assembly listing, whose loop-depth
    annotations locate the Gray loop."""
    build = pytest.importorskip("paper_2503_21596_amd._build")
    if not os.path.exists(build.HIPCC):
        pytest.skip("hipcc not found")
    src = os.path.join(build.CSRC, "ld_kernels_dary_s.hip")
    parts = [u for u in build.UNITS if u[0] == "ld_kernels_dary_s.hip"]
    assert parts

    def listing(unit):
        d = tmp_path / unit[2]
        d.mkdir()
        cmd = [build.HIPCC] + build.COMMON + build.DEVICE + unit[1] + ["-x", "hip", "-c", src, "-o",
                                                                       str(d / "kds.o"), "--save-temps"]
        subprocess.run(cmd, check=True, capture_output=True, cwd=d)
        names = [f for f in os.listdir(d) if f.endswith(".s") and "gfx950" in f]
        assert len(names) == 1, os.listdir(d)
        return gray_loop_spills(open(d / names[0]).read().splitlines())

    with concurrent.futures.ThreadPoolExecutor(max_workers=len(parts)) as ex:
        found = list(ex.map(listing, parts))
    spills = {}
    for f in found:
        assert not set(f) & set(spills), "an instantiation in two parts"
        spills.update(f)
    # 32-bit: d = 3 at 4 .. 52 columns, d = 4 at 4 .. 40; packed: d = 3 at 2 .. 32
    # dwords, d = 4 at 2 .. 24, each with two low-row counts (5 and 4 for d = 3, 4
    # and 3 for d = 4)
    assert len([k for k in spills if k[0] == 32]) == 23, sorted(spills)
    packed = [k for k in spills if k[0] == 16]
    assert len(packed) == 56, sorted(spills)
    assert {k[3] for k in packed if k[2] == 3} == {4, 5} and {k[3] for k in packed if k[2] == 4} == {3, 4}
    assert all(v == 0 for v in spills.values()), {k: v for k, v in spills.items() if v}


# ---------------------------------------------------------------------------
# 4. Queue pops: every wave takes its next item index from a returning atomic
# and broadcasts it with v_readfirstlane.  That is only sound when the lane that
# v_readfirstlane reads is the lane that performed the atomic.  The compiler's own
# atomic optimizer guarantees it: it guards the atomic with "first active lane"
# (v_mbcnt of exec compared with 0) and broadcasts after restoring the same exec.
# A hand-written "lane 0 only" guard does not: if the wave reaches that code with
# lane 0 inactive, v_readfirstlane reads a lane that never performed the atomic
# (a stale index), and the wave can loop forever.  The scan flags every returning
# atomic whose result reaches v_readfirstlane under a guard other than the
# first-active-lane one, or with exec narrowed further in between.

RET_ATOMIC = re.compile(r"\s+(global|flat|buffer)_atomic_\w+\s+v(\d+)(?:,|\s).*\bsc0\b")
READFIRST = re.compile(r"\s+v_readfirstlane_b32\s+s\d+,\s+v(\d+)\b")
SAVEEXEC = re.compile(r"\s+s_and_saveexec_b64\s+s\[(\d+):(\d+)\],\s+vcc")
RESTORE = re.compile(r"\s+s_or_b64\s+exec,\s+exec,\s+s\[(\d+):(\d+)\]")
CMP_LANE0 = re.compile(r"\s+v_cmp_eq_u32_e32\s+vcc,\s+0,\s+v(\d+)\b")
VDST = re.compile(r"\s+(v_\w+)\s+v(\d+),")


def unsafe_broadcasts(lines, checked=None):
    """(function, line) of v_readfirstlane reads of a returning atomic's result
    that are not guaranteed to read the lane that performed the atomic.  `checked`
    (a list) receives every such broadcast found, safe or not."""
    bad = []
    fn = None
    writer = {}        # VGPR -> opcode that last wrote it
    guard_src = None   # kind of the last vcc = (v == 0) compare: "first" or "other"
    stack = []         # open exec-narrowing regions: (saved sgpr pair, kind)
    atom = {}          # VGPR -> (kind of the innermost guard, depth of the stack) at the atomic
    for line in lines:
        f = FUNC.match(line)
        if f:
            fn, writer, guard_src, stack, atom = f.group(1), {}, None, [], {}
            continue
        s = line.split("//")[0]
        m = CMP_LANE0.match(s)
        if m:
            guard_src = "first" if writer.get(int(m.group(1))) == "v_mbcnt_hi_u32_b32" else "other"
        elif "vcc" in s.split(",")[0] and s.strip().startswith("v_cmp"):
            guard_src = "other"
        m = SAVEEXEC.match(s)
        if m:
            stack.append((m.group(1), guard_src or "other"))
            continue
        m = RESTORE.match(s)
        if m:
            for i in range(len(stack) - 1, -1, -1):
                if stack[i][0] == m.group(1):
                    del stack[i:]
                    break
            continue
        m = RET_ATOMIC.match(s)
        if m:
            atom[int(m.group(2))] = (stack[-1][1] if stack else "none", len(stack))
            continue
        m = READFIRST.match(s)
        if m and int(m.group(1)) in atom:
            kind, depth = atom.pop(int(m.group(1)))
            if checked is not None:
                checked.append((fn, kind))
            if kind == "other" or (kind == "first" and len(stack) != depth - 1) or \
                    (kind == "none" and len(stack) != depth):
                bad.append((fn, s.strip()))
            continue
        m = VDST.match(s)
        if m:
            writer[int(m.group(2))] = m.group(1)
            atom.pop(int(m.group(2)), None)
    return bad


def test_broadcast_scan_catches_a_lane0_guard():
    """The pattern of a lane-0-only pop (the compiler may re-enter the loop with
    lane 0 inactive) is flagged; the atomic optimizer's first-active-lane form is
    not."""
    bad = ["0000000000000000 <k>:",
           "\tv_and_b32_e32 v7, 63, v0",
           "\tv_cmp_eq_u32_e32 vcc, 0, v7",
           "\ts_and_saveexec_b64 s[0:1], vcc",
           "\tglobal_atomic_add v2, v1, v2, s[4:5] sc0",
           "\ts_or_b64 exec, exec, s[0:1]",
           "\ts_waitcnt vmcnt(0)",
           "\tv_readfirstlane_b32 s0, v2"]
    assert len(unsafe_broadcasts(bad)) == 1
    good = list(bad)
    good[1:2] = ["\tv_mbcnt_lo_u32_b32 v7, exec_lo, 0", "\tv_mbcnt_hi_u32_b32 v7, exec_hi, v7"]
    assert unsafe_broadcasts(good) == []
    # exec narrowed again before the broadcast
    worse = good[:-1] + ["\tv_cmp_gt_u32_e32 vcc, 5, v9", "\ts_and_saveexec_b64 s[8:9], vcc", good[-1]]
    assert len(unsafe_broadcasts(worse)) == 1


@pytest.mark.parametrize("obj", ["kbin0.o", "kbin1.o", "kbin2.o", "kdary.o", "kdarys0.o", "kdarys1.o", "kdarys2.o", "kdarys3.o", "kmfma0.o", "kmfma1.o",
                                 "kmfma2.o"])
def test_queue_pops_broadcast_the_atomic_lane(obj, tmp_path):
    path = os.path.join(BUILD, obj)
    if not os.path.exists(path):
        pytest.skip("library not built (run __graft_entry__.build())")
    if not os.path.exists(f"{LLVM}/llvm-objdump"):
        pytest.skip("ROCm LLVM tools not found")
    lines = _disassemble(path, tmp_path)
    checked = []
    bad = unsafe_broadcasts(lines, checked)
    # every queue kernel pops through one (the d-ary SGPR-operand unit is built in
    # four parts, each with a quarter of its kernels)
    assert len(checked) > (20 if obj.startswith("kdarys") else 40), len(checked)
    assert not bad, bad[:5]
