"""Static check of the built gfx950 code for the wait states that software
must provide (CDNA3/CDNA4 instruction-set reference, "manually inserted wait
states").  The compiler inserts them for the instructions it emits, but not
for instructions written in inline asm: the DPP broadcasts, masked selects and
lane writes of the kernels carry their own `s_nop`s, and this module checks,
on the disassembly of the library's own code objects, that every such hazard
is covered on every control-flow path.

Rules checked (writer -> reader: independent wait states required between):
  dpp_src      VALU writes a VGPR -> a DPP instruction reads it as src0:   2
  dpp_exec     VALU writes EXEC (v_cmpx) -> any DPP instruction:          5
  trans_use    transcendental op (v_rcp, v_rsq, v_sqrt, v_exp, v_log,
               v_sin, v_cos) writes a VGPR -> a non-transcendental VALU
               instruction reads it:                                       1
  lane_select  VALU writes an SGPR -> v_readlane / v_writelane takes it as
               the lane select:                                            4
  mfma_dpp     MFMA writes a VGPR -> a DPP instruction reads it: at least
               as many as the compiler leaves before the plain VALU readers
               of the same MFMA opcode anywhere in the build (its own
               hazard table, which inline asm does not get).

Each instruction counts one wait state, `s_nop N` counts N + 1.  Paths follow
fall-through and branch edges inside a function.

Test infrastructure only: reads the built shared library, never the GPU.
"""
from __future__ import annotations

import collections
import os
import re
import struct
import subprocess
import tempfile

LLVM = "/opt/rocm/llvm/bin"
BUNDLE_MAGIC = b"__CLANG_OFFLOAD_BUNDLE__"

_INS = re.compile(r"^\t(\S+)\s*(.*?)\s*//\s*([0-9A-F]+):")
_FN = re.compile(r"^([0-9a-f]+) <(.+)>:$")
_TGT = re.compile(r"<(.+)\+0x([0-9a-f]+)>\s*$")
_UNCOND = ("s_branch", "s_setpc_b64", "s_endpgm")
_TRANS = ("v_rcp_", "v_rsq_", "v_sqrt_", "v_exp_", "v_log_", "v_sin_", "v_cos_")

Ins = collections.namedtuple("Ins", "mn ops addr target")


def code_objects(so_path: str, outdir: str, arch: str = "gfx950") -> list[str]:
    """Write every `arch` code object bundled in the library's .hip_fatbin
    section (one clang offload bundle per linked object) to outdir."""
    fb = os.path.join(outdir, "fatbin.bin")
    subprocess.run([os.path.join(LLVM, "llvm-objcopy"), f"--dump-section=.hip_fatbin={fb}", so_path,
                    os.path.join(outdir, "copy.so")], check=True, capture_output=True)
    data = open(fb, "rb").read()
    paths, pos = [], 0
    while (i := data.find(BUNDLE_MAGIC, pos)) >= 0:
        (count,) = struct.unpack_from("<Q", data, i + len(BUNDLE_MAGIC))
        p = i + len(BUNDLE_MAGIC) + 8
        for _ in range(count):
            off, size, tlen = struct.unpack_from("<QQQ", data, p)
            p += 24
            triple = data[p:p + tlen].decode()
            p += tlen
            if triple.endswith(arch):
                path = os.path.join(outdir, f"co{len(paths)}.o")
                with open(path, "wb") as f:
                    f.write(data[i + off:i + off + size])
                paths.append(path)
        pos = i + 1
    return paths


def disassemble(co_path: str) -> str:
    r = subprocess.run([os.path.join(LLVM, "llvm-objdump"), "-d", "--no-show-raw-insn", co_path],
                       check=True, capture_output=True, text=True)
    return r.stdout


def kernel_meta(co_path: str) -> dict[str, dict[str, int]]:
    """Kernel symbol -> its integer metadata fields (.vgpr_count,
    .private_segment_fixed_size, .vgpr_spill_count, ...) from the code
    object's metadata note."""
    r = subprocess.run([os.path.join(LLVM, "llvm-readelf"), "--notes", co_path],
                       check=True, capture_output=True, text=True)
    blocks, cur = [], {}
    for line in r.stdout.splitlines():
        if re.match(r"\s+- \.", line):  # a new kernel's entry
            cur = {}
            blocks.append(cur)
        m = re.match(r"\s+-?\s*\.([a-z_]+):\s+(\S+)", line)
        if m:
            cur[m.group(1)] = m.group(2)
    out = {}
    for b in blocks:
        if "name" in b and "vgpr_count" in b:
            out[b["name"]] = {k: int(v) for k, v in b.items() if v.lstrip("-").isdigit()}
    return out


def kernel_vgprs(co_path: str) -> dict[str, int]:
    """Kernel symbol -> .vgpr_count."""
    return {k: v["vgpr_count"] for k, v in kernel_meta(co_path).items()}


def parse(text: str) -> list[dict]:
    """Functions of an llvm-objdump listing: name, base address, instructions."""
    funcs, cur = [], None
    for line in text.splitlines():
        m = _FN.match(line)
        if m:
            cur = {"name": m.group(2), "base": int(m.group(1), 16), "ins": []}
            funcs.append(cur)
            continue
        m = _INS.match(line)
        if m and cur is not None:
            t = _TGT.search(line)
            tgt = None
            if t and t.group(1) == cur["name"]:
                tgt = cur["base"] + int(t.group(2), 16)
            cur["ins"].append(Ins(m.group(1), m.group(2), int(m.group(3), 16), tgt))
    return funcs


def operands(ops: str) -> list[str]:
    """The comma-separated operands, without trailing DPP / modifier words."""
    out = []
    for p in re.split(r",\s*", ops):
        w = p.split()
        if w:
            out.append(w[0])
    return out


def regs(tok: str, kind: str = "v") -> set[int]:
    """Register numbers of one operand of the given kind ('v' VGPR, 's' SGPR)."""
    tok = tok.strip().lstrip("-").strip("|")
    tok = re.sub(r"^(neg|abs)\((.*)\)$", r"\2", tok)
    m = re.match(rf"^{kind}(\d+)$", tok)
    if m:
        return {int(m.group(1))}
    m = re.match(rf"^{kind}\[(\d+):(\d+)\]$", tok)
    if m:
        return set(range(int(m.group(1)), int(m.group(2)) + 1))
    return set()


_CARRY_OUT = ("v_add_co_", "v_sub_co_", "v_subrev_co_", "v_addc_co_", "v_subb_co_", "v_subbrev_co_",
              "v_div_scale_", "v_mad_u64_u32", "v_mad_i64_i32")


class Info:
    """What one instruction writes and reads (register sets) and its wait states."""
    __slots__ = ("dpp", "vw", "vr", "src0", "sw", "lsel", "ws", "trans", "mfma", "valu", "cmpx")

    def __init__(self, i: Ins):
        mn = i.mn
        o = operands(i.ops)
        self.valu = mn.startswith("v_")
        self.dpp = "_dpp" in mn
        self.trans = mn.startswith(_TRANS)
        self.mfma = mn.startswith("v_mfma")
        self.cmpx = mn.startswith("v_cmpx")
        self.ws = int(i.ops.split()[0], 0) + 1 if mn == "s_nop" else 1
        self.vw = set()
        self.vr = set()
        self.sw = set()
        self.lsel = set()
        self.src0 = regs(o[1]) if self.dpp and len(o) > 1 else set()
        if not self.valu or not o:
            return
        for x in o[1:]:
            self.vr |= regs(x)
        if mn.startswith(("v_fmac", "v_mac")):
            self.vr |= regs(o[0])
        if not mn.startswith(("v_readlane", "v_readfirstlane", "v_cmp")):
            self.vw = regs(o[0])
            if mn.startswith(("v_swap_b32", "v_permlane")) and len(o) > 1:
                self.vw |= regs(o[1])
        # SGPR / VCC destinations: the first operand (v_readlane, VOPC), and
        # the carry-out second operand of the VOP3b forms
        dst = [o[0]] + ([o[1]] if mn.startswith(_CARRY_OUT) and len(o) > 1 else [])
        for x in dst:
            self.sw |= regs(x, "s") | ({"vcc"} if x.startswith("vcc") else set())
        if mn.startswith("v_cmp") and mn.endswith("_e32"):
            self.sw |= {"vcc"}
        if mn.startswith(("v_readlane_b32", "v_writelane_b32")) and len(o) > 2:
            self.lsel = regs(o[2], "s") | ({"vcc"} if o[2].startswith("vcc") else set())


class Function:
    def __init__(self, f: dict):
        self.name, self.ins = f["name"], f["ins"]
        self.info = [Info(i) for i in self.ins]
        idx = {ins.addr: k for k, ins in enumerate(self.ins)}
        self.succ = []
        for k, ins in enumerate(self.ins):
            s = []
            if ins.mn not in _UNCOND and k + 1 < len(self.ins):
                s.append(k + 1)
            if ins.target is not None and (ins.mn == "s_branch" or ins.mn.startswith("s_cbranch")):
                if ins.target in idx:
                    s.append(idx[ins.target])
            self.succ.append(s)

    def readers_within(self, k: int, need: int, pred) -> list[tuple[int, int]]:
        """Instructions j reachable from k at fewer than `need` wait states
        for which pred(info of j) holds: (j, wait states between k and j)."""
        best, out = {}, []
        stack = [(j, 0) for j in self.succ[k]]
        info, succ = self.info, self.succ
        while stack:
            j, d = stack.pop()
            if d >= need or best.get(j, need) <= d:
                continue
            best[j] = d
            if pred(info[j]):
                out.append((j, d))
            dd = d + info[j].ws
            for s in succ[j]:
                stack.append((s, dd))
        return out


def check(funcs: list[dict], mfma_dpp_need: int | None = None, mfma_search: int = 24) -> dict:
    """Run every rule; returns {'violations': [(rule, function, writer,
    reader, wait states)], 'counts': Counter, 'mfma_valu_min': {opcode: the
    fewest wait states the compiler leaves before a plain VALU reader}}."""
    fns = [Function(f) for f in funcs]
    viol, counts = [], collections.Counter()
    mfma_min: dict[str, int] = {}
    for fn in fns:  # calibrate the MFMA rule on the compiler's own readers
        for k, inf in enumerate(fn.info):
            if inf.mfma:
                w = inf.vw
                hits = fn.readers_within(k, mfma_search, lambda r: r.valu and not r.mfma and not r.dpp and bool(r.vr & w))
                for _, d in hits:
                    mn = fn.ins[k].mn
                    mfma_min[mn] = min(mfma_min.get(mn, mfma_search), d)
    for fn in fns:
        for k, inf in enumerate(fn.info):
            counts["dpp"] += inf.dpp
            counts["lane_select"] += bool(inf.lsel)
            w = inf.vw
            hits = []
            if w:
                hits += [("dpp_src", j, d) for j, d in fn.readers_within(k, 2, lambda r: r.dpp and bool(r.src0 & w))]
                if inf.trans:
                    counts["trans"] += 1
                    hits += [("trans_use", j, d) for j, d in
                             fn.readers_within(k, 1, lambda r: r.valu and not r.trans and bool(r.vr & w))]
                if inf.mfma:
                    counts["mfma"] += 1
                    need = mfma_dpp_need if mfma_dpp_need is not None else mfma_min.get(fn.ins[k].mn, 0)
                    hits += [("mfma_dpp", j, d) for j, d in fn.readers_within(k, need, lambda r: r.dpp and bool(r.vr & w))]
            if inf.cmpx:
                hits += [("dpp_exec", j, d) for j, d in fn.readers_within(k, 5, lambda r: r.dpp)]
            sw = inf.sw
            if sw:
                hits += [("lane_select", j, d) for j, d in fn.readers_within(k, 4, lambda r: bool(r.lsel & sw))]
            viol += [(rule, fn.name, fn.ins[k], fn.ins[j], d) for rule, j, d in hits]
    return {"violations": viol, "counts": counts, "mfma_valu_min": mfma_min}


def scan_library(so_path: str) -> tuple[list[dict], dict[str, dict[str, int]]]:
    """Parsed functions and kernel metadata of every gfx950 code object."""
    funcs, meta = [], {}
    with tempfile.TemporaryDirectory() as tmp:
        for co in code_objects(so_path, tmp):
            funcs += parse(disassemble(co))
            meta.update(kernel_meta(co))
    return funcs, meta
