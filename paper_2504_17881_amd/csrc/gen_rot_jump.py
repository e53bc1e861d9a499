#!/usr/bin/env python3
"""Writes rot_jump_f32m4.inc: the complex64, rank-4 static-sign rotation
variants as one inline-assembly jump table.

A static-sign rotation on a thread's 16 amplitudes is one of 64 variants,
var = slot * 16 + imag * 8 + zp (slot: the basis direction I of the
rotation's x; imag: tau imaginary; zp: the sign pattern's 3 bits).  Variant
var updates the 8 pairs (v, v | 2^I) with the two-FMA in-place pair update,
negating both coefficients of a pair when parity(drop_bit(v, I) & zp) is
odd.  Every variant is 32 v_fma_f32 (8 bytes each) and one s_branch (4
bytes): 260 bytes, so the block jumps straight to byte offset 260 * var of
its table instead of walking a branch tree.

Operands of the generated block: %0..%31 the amplitudes (re, im of amp[0],
amp[1], ...), %32 a scratch SGPR, %33 ga, %34 gb, %35 var; it clobbers
s[90:91] and SCC.  rot_jump_f64m4.inc is the same table for complex128:
the same layout with v_fma_f64 on register pairs (also 8 bytes each).

It also writes rot_loop_f32m4.inc: a whole run of rotations of a tile
chunk as one block of threaded code.  A header loads the first 32-byte
rotation record with one scalar load, computes the lane's sign and the two
coefficients and jumps to its variant.  Each variant issues the load of the
next record, applies its 32 FMAs, and then does the same dispatch for the
next record itself, jumping straight to that record's variant: a rotation
takes one computed jump and no other taken branch, and the record's load
overlaps the FMAs (the table must be followed by 32 readable bytes).  The
block is left, without consuming it, at a diagonal record (var = 64; the
caller applies it) and at the end of the run.  Variants are 380 bytes:
the load (8), 32 v_fma_f32, the count test and exit (8), the wait (4) and
the dispatch (112).  Operands: %0..%31 the amplitudes, %[plo], %[phi] the
record pointer and %[cnt] the records left (read and written), %[ga], %[gb]
scratch, %[k0] the lane's coset representative, %[tb] the base tile index;
it clobbers s[76:91] and SCC.

rot_loop_f64m4.inc is the threaded loop for complex128: 40-byte records
(tau_b at byte 32, loaded into s[92:93]), v_fma_f64 on register pairs, and
the lane's sign applied as a factor of +-1.0 (v_cvt_f64_i32 of 1 - 2 parity)
by two v_mul_f64, since the high word of a register pair operand cannot be
named on its own; variants are 404 bytes and the table must be followed by
40 readable bytes.  Extra operands: %[sg] (a register pair) and %[t]
scratch; it also clobbers s[92:93].

Run from this directory: python3 gen_rot_jump.py
"""
import os

M = 4
VARIANT_BYTES = 32 * 8 + 4
LOOP_VARIANT_BYTES = 32 * 8 + 124


def drop_bit(v, i):
    return ((v >> (i + 1)) << i) | (v & ((1 << i) - 1))


def pair(v, w, imag, neg, ga="%33", gb="%34", op="v_fma_f32"):
    ar, ai, br, bi = f"%{2 * v}", f"%{2 * v + 1}", f"%{2 * w}", f"%{2 * w + 1}"
    n = "-" if neg else ""
    p = "" if neg else "-"
    if not imag:
        return [f"{op} {ar}, {n}{ga}, {br}, {ar}",
                f"{op} {ai}, {n}{ga}, {bi}, {ai}",
                f"{op} {br}, {n}{gb}, {ar}, {br}",
                f"{op} {bi}, {n}{gb}, {ai}, {bi}"]
    # a <- a + i ga b, b <- b + i gb a (negated coefficients when neg)
    return [f"{op} {ar}, {p}{ga}, {bi}, {ar}",
            f"{op} {ai}, {n}{ga}, {br}, {ai}",
            f"{op} {br}, {p}{gb}, {ai}, {br}",
            f"{op} {bi}, {n}{gb}, {ar}, {bi}"]


def fmas(var, ga="%33", gb="%34", op="v_fma_f32"):
    slot, imag, zp = var >> M, (var >> (M - 1)) & 1, var & ((1 << (M - 1)) - 1)
    out = []
    for v in range(1 << M):
        if v >> slot & 1:
            continue
        neg = bin(drop_bit(v, slot) & zp).count("1") & 1
        out += pair(v, v | (1 << slot), imag, neg, ga, gb, op)
    assert len(out) == 32
    return out


def variant(var, op="v_fma_f32"):
    return fmas(var, op=op) + ["s_branch 3f"]


def block(op="v_fma_f32"):
    lines = ["s_min_u32 %32, %35, 63",
             f"s_mul_i32 %32, %32, {VARIANT_BYTES}",
             "s_getpc_b64 s[90:91]",
             "1:",
             "s_add_u32 s90, s90, %32",
             "s_addc_u32 s91, s91, 0",
             "s_add_u32 s90, s90, (2f - 1b)",
             "s_addc_u32 s91, s91, 0",
             "s_setpc_b64 s[90:91]",
             "2:"]
    for var in range(M << M):
        lines += variant(var, op)
    lines.append("3:")
    return lines


# the header that computes the lane's coefficients for the record at s[80:87]
# and jumps to its variant; `off` is the assembler expression for the table
# start minus the address after s_getpc_b64, `hi` the high-word carry term
def _dispatch(off, hi):
    return ["s_bfe_u32 s88, s84, 0x80010",    # var = info bits 16..23
            "s_cmp_eq_u32 s88, 64",
            "s_cbranch_scc1 9f",              # diagonal: leave it to the caller
            "s_and_b64 s[82:83], s[82:83], %[tb]",
            "s_bcnt1_i32_b64 s89, s[82:83]",  # parity(tile & zhigh) in bit 0
            "v_and_b32 %[ga], s80, %[k0]",
            "v_bcnt_u32_b32 %[ga], %[ga], s89",
            "v_lshl_add_u32 %[gb], %[ga], 31, s87",
            "v_lshl_add_u32 %[ga], %[ga], 31, s86",
            "s_add_u32 s76, s76, 32",
            "s_addc_u32 s77, s77, 0",
            "s_sub_u32 s78, s78, 1",
            "s_min_u32 s88, s88, 63",
            f"s_mul_i32 s88, s88, {LOOP_VARIANT_BYTES}",
            "s_getpc_b64 s[90:91]",
            "1:",
            "s_add_u32 s90, s90, s88",
            "s_addc_u32 s91, s91, 0",
            f"s_add_u32 s90, s90, {off}",
            f"s_addc_u32 s91, s91, {hi}",
            "s_setpc_b64 s[90:91]"]


def loop_block():
    lines = ["s_mov_b32 s76, %[plo]",          # record pointer and count in
             "s_mov_b32 s77, %[phi]",          # fixed registers
             "s_mov_b32 s78, %[cnt]",
             "s_cmp_eq_u32 s78, 0",
             "s_cbranch_scc1 9f",
             "s_load_dwordx8 s[80:87], s[76:77], 0x0",
             "s_waitcnt lgkmcnt(0)"] + _dispatch("(2f - 1b)", "0") + ["2:"]
    for var in range(M << M):
        # the next record's load is issued before the FMAs (the table is
        # followed by readable padding), its dispatch after them
        lines += (["s_load_dwordx8 s[80:87], s[76:77], 0x0"] + fmas(var, "%[ga]", "%[gb]") +
                  ["s_cmp_eq_u32 s78, 0", "s_cbranch_scc1 9f", "s_waitcnt lgkmcnt(0)"] +
                  _dispatch("(2b - 1b)", "-1"))
    lines += ["9:", "s_mov_b32 %[plo], s76", "s_mov_b32 %[phi], s77", "s_mov_b32 %[cnt], s78"]
    return lines


# complex128: 40-byte records (tau_b at byte 32 in s[92:93]); the lane sign
# becomes a factor of +-1.0 that multiplies both coefficients
LOOP64_VARIANT_BYTES = 404


def _dispatch64(off, hi):
    return ["s_bfe_u32 s88, s84, 0x80010",
            "s_cmp_eq_u32 s88, 64",
            "s_cbranch_scc1 9f",
            "s_and_b64 s[82:83], s[82:83], %[tb]",
            "s_bcnt1_i32_b64 s89, s[82:83]",
            "v_and_b32 %[t], s80, %[k0]",
            "v_bcnt_u32_b32 %[t], %[t], s89",
            "v_and_b32 %[t], 1, %[t]",
            "v_mad_i32_i24 %[t], %[t], -2, 1",     # 1 - 2 parity
            "v_cvt_f64_i32 %[sg], %[t]",
            "v_mul_f64 %[ga], %[sg], s[86:87]",
            "v_mul_f64 %[gb], %[sg], s[92:93]",
            "s_add_u32 s76, s76, 40",
            "s_addc_u32 s77, s77, 0",
            "s_sub_u32 s78, s78, 1",
            "s_min_u32 s88, s88, 63",
            f"s_mul_i32 s88, s88, {LOOP64_VARIANT_BYTES}",
            "s_getpc_b64 s[90:91]",
            "1:",
            "s_add_u32 s90, s90, s88",
            "s_addc_u32 s91, s91, 0",
            f"s_add_u32 s90, s90, {off}",
            f"s_addc_u32 s91, s91, {hi}",
            "s_setpc_b64 s[90:91]"]


def loop_block64():
    loads = ["s_load_dwordx8 s[80:87], s[76:77], 0x0",
             "s_load_dwordx2 s[92:93], s[76:77], 0x20"]
    lines = (["s_mov_b32 s76, %[plo]", "s_mov_b32 s77, %[phi]", "s_mov_b32 s78, %[cnt]",
              "s_cmp_eq_u32 s78, 0", "s_cbranch_scc1 9f"] + loads +
             ["s_waitcnt lgkmcnt(0)"] + _dispatch64("(2f - 1b)", "0") + ["2:"])
    for var in range(M << M):
        lines += (loads + fmas(var, "%[ga]", "%[gb]", "v_fma_f64") +
                  ["s_cmp_eq_u32 s78, 0", "s_cbranch_scc1 9f", "s_waitcnt lgkmcnt(0)"] +
                  _dispatch64("(2b - 1b)", "-1"))
    lines += ["9:", "s_mov_b32 %[plo], s76", "s_mov_b32 %[phi], s77", "s_mov_b32 %[cnt], s78"]
    return lines


def main():
    here = os.path.dirname(os.path.abspath(__file__))
    text = ("// Generated by gen_rot_jump.py; do not edit.\n"
            "// Jump table of the 64 complex64 rank-4 static-sign rotation variants\n"
            "// (operands and layout: see gen_rot_jump.py).\n"
            "#pragma once\n"
            f"#define PRX_ROT_JUMP_VARIANT_BYTES {VARIANT_BYTES}\n"
            "#define PRX_ROT_JUMP_F32M4 \\\n" + " \\\n".join(
                f'    "{line}\\n"' for line in block()) + "\n")
    with open(os.path.join(here, "rot_jump_f32m4.inc"), "w") as f:
        f.write(text)
    text = ("// Generated by gen_rot_jump.py; do not edit.\n"
            "// Jump table of the 64 complex128 rank-4 static-sign rotation variants\n"
            "// (v_fma_f64 on register pairs; operands and layout as the complex64\n"
            "// table: see gen_rot_jump.py).\n"
            "#pragma once\n"
            "#define PRX_ROT_JUMP_F64M4 \\\n" + " \\\n".join(
                f'    "{line}\\n"' for line in block("v_fma_f64")) + "\n")
    with open(os.path.join(here, "rot_jump_f64m4.inc"), "w") as f:
        f.write(text)
    text = ("// Generated by gen_rot_jump.py; do not edit.\n"
            "// Threaded rotation loop over the 64 complex64 rank-4 static-sign\n"
            "// variants (operands and layout: see gen_rot_jump.py).\n"
            "#pragma once\n"
            f"#define PRX_ROT_LOOP_VARIANT_BYTES {LOOP_VARIANT_BYTES}\n"
            "#define PRX_ROT_LOOP_F32M4 \\\n" + " \\\n".join(
                f'    "{line}\\n"' for line in loop_block()) + "\n")
    with open(os.path.join(here, "rot_loop_f32m4.inc"), "w") as f:
        f.write(text)
    text = ("// Generated by gen_rot_jump.py; do not edit.\n"
            "// Threaded rotation loop over the 64 complex128 rank-4 static-sign\n"
            "// variants (operands and layout: see gen_rot_jump.py).\n"
            "#pragma once\n"
            f"#define PRX_ROT_LOOP64_VARIANT_BYTES {LOOP64_VARIANT_BYTES}\n"
            "#define PRX_ROT_LOOP_F64M4 \\\n" + " \\\n".join(
                f'    "{line}\\n"' for line in loop_block64()) + "\n")
    with open(os.path.join(here, "rot_loop_f64m4.inc"), "w") as f:
        f.write(text)


if __name__ == "__main__":
    main()
