"""Generate the gfx950 dispatch loop of the float32 interpreter.

Writes dispatch_f32.inc: for each (K, S) in VARIANTS two device functions,
run_f32_dispatch_K_S() (branch-table dispatch) and run_f32d_dispatch_K_S()
(direct dispatch into handler slots), each holding one inline-asm block that
runs one chunk's program and stores the chunk's value; and dispatch_bool.inc,
the Boolean loops.

Why assembly: the interpreter spends most of its scalar instructions on
choosing the handler.  The compiler lowers a switch to a tree of compares
(about nine compare-and-branch pairs per instruction word); here the word's
10-bit key indexes a table of branches, so choosing the handler costs five
scalar instructions and one branch.  Each handler ends with the code that
fetches the next-but-one word and jumps to the next word's handler.

Register plan (per lane): st[d][k] = v[V_ST + d*K + k], x[k] = v[V_X + k],
q[k] = PDIV(x[k], x[k]) at v[V_Q + k], the refined reciprocal of x[k] at
v[V_Y + k], five temporaries from V_T; scalar temporaries from S_BASE, per k
the lane mask |x[k]| < 1e-6, the bounds of the short divides and a flag word
saying which short divides this chunk's x allows.  All of them are declared
clobbered, so the compiler keeps its own values elsewhere.

Work that depends on x alone does not change while a chunk runs, so it is
done once per chunk: the protected quotient x/x (a handler whose operands
are both x then only copies it), the protection mask used when x is the
divisor, the refined reciprocal of x and the range flags below.

Memory: every load issued here is waited for inside the block (no value is
left in flight when the block ends); PUSH, LOAD and STORE address exactly the
slots the C++ interpreter addresses.  The word kEndWord ends every chunk and
every other key leads to a handler that moves to the next word, so the loop
always reaches the end of the chunk's code.

The protected divide is the instruction sequence the compiler emits for an
IEEE float division with denormals enabled (div_scale, rcp, two Newton steps,
div_fmas, div_fixup), in the same order, followed by the select of 1.0 where
|b| < 1e-6; the wait states between dependent instructions are the
compiler's (rcp result used two instructions later, VCC written six
instructions before div_fmas reads it, the mask written twelve instructions
before the select reads it).

Short divides.  When neither operand nor any intermediate of that sequence
can leave the normal range, div_scale returns its operand unchanged with VCC
clear, div_fmas is a plain fma and div_fixup returns its first operand: the
remaining steps (rcp, the two Newton steps, the final fma) give the same bits.
The short form then stops one step earlier, by Markstein's theorem (Handbook
of Floating-Point Arithmetic, on division by FMA): if y is the correctly
rounded 1/b and q is within one ulp of a/b, the residual r = a - b*q is exact
and q + r*y rounded to nearest is the correctly rounded a/b.  Here y = rcp(b)
refined by one Newton step, and on this hardware that y equals the correctly
rounded 1/b for every divisor with |b| in [2^-21, 2^65) (an exhaustive check
of all 1.44e9 of them); q = a*y.  So the short form is rcp, two steps for y,
the product, the residual and one correction (5 instructions per case after
the rcp, 3 when y is hoisted).  On both short-divide domains it matched IEEE
division on 1.7e10 random quotients and on 2.6e9 quotients built to lie
within 63 * 2^-48 (relative) of a rounding midpoint, where the same step with
the unrefined rcp(b) fails about once in 2400.  Because q = a*y can be up to
1.5 ulp from a/b, outside the theorem's hypothesis, the short form is also
checked exhaustively over every numerator significand for sampled divisor
significands (tests/csrc/short_divide_check.c).
Two kinds of handler use this:
  * stack / x: the refined reciprocal of x is hoisted with the other x-only
    work.  Allowed when every lane's unprotected x lies in [1e-6, 2^20] (a
    per-chunk flag) and every numerator lies in [2^-90, 2^70]: the quotient
    stays in [2^-110, 2^90], each residual a - x*q is a multiple of 2^-137 and
    so exact, and the exponent gap stays below the 96 at which div_scale
    would rescale.
  * x / stack: allowed when every lane's x lies in [2^-60, 2^60] (a per-chunk
    flag) and every divisor satisfies |b| <= 2^64: an unprotected divisor is
    then in [1e-6, 2^64], the quotient in [2^-124, 2^80] and the reciprocal
    normal.
  * stack / stack: the x / stack argument with the numerator's range checked
    per case instead of per chunk: every |numerator| in [2^-60, 2^60] and
    every |divisor| <= 2^64.
Where no lane's divisor is protected (every |divisor| >= 1e-6: a per-chunk
flag for x, one more min-reduction for a stack value) the short form skips
the per-case protection compare and select.
Each check is made over all lanes and slots of the wave (a scalar branch):
the K values of a lane are reduced to their largest (and smallest) magnitude
with v_max3 / v_min3, then compared once.  Any value outside the ranges,
infinities included, sends the whole wave through the full sequence, and
protected lanes take 1.0 either way.  The reductions pass over a NaN (an IEEE
max/min returns the other operand), so a lane holding a NaN operand may take
the short form; every step of it propagates the NaN, so that lane's result is
NaN as the full sequence's is (payloads may differ; results are compared as
bit-equal or both NaN).
"""
from __future__ import annotations

import os
import sys

VARIANTS = [(4, 10), (8, 10)]
# A chunk's output vector is the one value that waves hand to each other
# inside a launch (the wave that finishes a chunk's last input reads it with
# LOAD).  It is written and read with agent-scope coherence (sc1, the form of
# a relaxed device-scope atomic store and load), and the chunk's end waits for
# its stores to complete before the kernel decrements the parent's counter.
# The counter update can then be relaxed: no L2 write-back before it and no
# L2 invalidation after it, so code, inputs and chunk headers stay cached.
SHARED = " sc1"
V_ST = 16
S_BASE = 64
M_XX, M_XS, M_SX, M_SS, M_RS, M_PUSH, M_LOAD, M_STORE = range(8)
END_KEY = 1 | (M_STORE << 2)          # kEndWord & 0x3ff
TINY = 0x358637BD                     # 1e-6f
P2 = lambda e: (127 + e) << 23        # bit pattern of 2^e (normal range)


def gen_one(K: int, S: int, direct: bool = False, SLOT: int = 128) -> str:
    """direct=False: the key indexes a table of branches to the handlers (two
    jumps per word).  direct=True: the key's slot of SLOT bytes at table +
    key * SLOT holds the handler itself for +, - and x (and the copy of x/x),
    so those words take one jump; divides, PUSH, LOAD and STORE stay out of
    line, one branch from their slot."""
    assert K % 2 == 0, "the range checks pair up slots"
    V_X = V_ST + S * K
    V_Q = V_X + K
    V_Y = V_Q + K
    V_T = V_Y + K
    V_CP = V_T + 5                    # destination of the code-line touches, read by nothing
    n_vgpr = V_CP + 1
    names = []
    for p in ["TB", "TG", "A", "J", "P"] + [f"XM{k}" for k in range(K)]:
        names += [f"{p}0", f"{p}1"]                   # pairs first: all even-aligned
    names += ["INS", "NXT", "OFF", "T0", "T1", "TINY", "FLG", "LOSX", "HISX", "HIXS"]
    s = {n: S_BASE + i for i, n in enumerate(names)}
    assert S_BASE % 2 == 0 and S_BASE + len(names) <= 100
    for k in range(K):
        s[f"XM{k}"] = s[f"XM{k}0"]
    sr = lambda n: f"s{s[n]}"
    sp = lambda n: f"s[{s[n]}:{s[n] + 1}]"
    st = lambda d, k: f"v{V_ST + d * K + k}"
    xv = lambda k: f"v{V_X + k}"
    T = [f"v{V_T + i}" for i in range(5)]
    L = []
    a = L.append

    def tail():
        a("  s_waitcnt lgkmcnt(0)")
        a(f"  s_mov_b32 {sr('INS')}, {sr('NXT')}")
        a(f"  s_add_u32 {sr('OFF')}, {sr('OFF')}, 4")
        a(f"  s_load_dword {sr('NXT')}, %[code], {sr('OFF')}")
        a(f"  s_and_b32 {sr('TG0')}, {sr('INS')}, 0x3ff")
        if direct:          # the slot of key k starts at table + k * SLOT
            a(f"  s_lshl_b32 {sr('TG0')}, {sr('TG0')}, {SLOT.bit_length() - 1}")
            a(f"  s_add_u32 {sr('TG0')}, {sr('TG0')}, {sr('TB0')}")
        else:               # entry k of the branch table
            a(f"  s_lshl2_add_u32 {sr('TG0')}, {sr('TG0')}, {sr('TB0')}")
        a(f"  s_addc_u32 {sr('TG1')}, {sr('TB1')}, 0")
        a(f"  s_setpc_b64 {sp('TG0')}")

    def op(f, dst, A, B, mask=None):
        if f == 0:
            a(f"  v_add_f32_e32 {dst}, {A}, {B}")
        elif f == 1:
            a(f"  v_sub_f32_e32 {dst}, {A}, {B}")
        elif f == 2:
            a(f"  v_mul_f32_e32 {dst}, {A}, {B}")
        else:
            if mask is None:
                a(f"  v_cmp_lt_f32_e64 {sp('P0')}, |{B}|, {sr('TINY')}")
                mask = sp('P0')
            a(f"  v_div_scale_f32 {T[0]}, {sp('J0')}, {B}, {B}, {A}")
            a(f"  v_rcp_f32_e32 {T[1]}, {T[0]}")
            a(f"  v_div_scale_f32 {T[2]}, vcc, {A}, {B}, {A}")
            a(f"  v_fma_f32 {T[3]}, -{T[0]}, {T[1]}, 1.0")
            a(f"  v_fmac_f32_e32 {T[1]}, {T[3]}, {T[1]}")
            a(f"  v_mul_f32_e32 {T[3]}, {T[2]}, {T[1]}")
            a(f"  v_fma_f32 {T[4]}, -{T[0]}, {T[3]}, {T[2]}")
            a(f"  v_fmac_f32_e32 {T[3]}, {T[4]}, {T[1]}")
            a(f"  v_fma_f32 {T[0]}, -{T[0]}, {T[3]}, {T[2]}")
            a(f"  v_div_fmas_f32 {T[0]}, {T[0]}, {T[1]}, {T[3]}")
            a(f"  v_div_fixup_f32 {T[0]}, {T[0]}, {B}, {A}")
            a(f"  v_cndmask_b32_e64 {dst}, {T[0]}, 1.0, {mask}")

    def reduce_abs(kind, dst, vals):
        """dst = max or min of |v| over vals (NaN operands are passed over,
        so a NaN lane takes the short divide too, where it also gives NaN)."""
        a(f"  v_{kind}3_f32 {dst}, |{vals[0]}|, |{vals[1]}|, |{vals[2]}|")
        i = 3
        while i + 1 < len(vals):
            a(f"  v_{kind}3_f32 {dst}, {dst}, |{vals[i]}|, |{vals[i + 1]}|")
            i += 2
        if i < len(vals):
            a(f"  v_{kind}_f32_e64 {dst}, {dst}, |{vals[i]}|")

    def short_div(dst, num, den, protect=True):
        """The short divide (see the module docstring): the refined reciprocal
        y, q = num * y, one correction q + (num - den * q) * y; then 1.0 where
        |den| < 1e-6 (protect=False: no lane has such a den)."""
        a(f"  v_rcp_f32_e32 {T[1]}, {den}")
        if protect:
            a(f"  v_cmp_lt_f32_e64 {sp('P0')}, |{den}|, {sr('TINY')}")
        else:
            a("  s_nop 0")                    # a transcendental's result is read one instruction later
        a(f"  v_fma_f32 {T[3]}, -{den}, {T[1]}, 1.0")
        a(f"  v_fmac_f32_e32 {T[1]}, {T[3]}, {T[1]}")
        a(f"  v_mul_f32_e32 {T[3]}, {num}, {T[1]}")
        a(f"  v_fma_f32 {T[4]}, -{den}, {T[3]}, {num}")
        if protect:
            a(f"  v_fma_f32 {T[0]}, {T[4]}, {T[1]}, {T[3]}")
            a(f"  v_cndmask_b32_e64 {dst}, {T[0]}, 1.0, {sp('P0')}")
        else:
            a(f"  v_fma_f32 {dst}, {T[4]}, {T[1]}, {T[3]}")

    def short_div_both(name, dsts, nums, dens):
        """Both forms of the short divide: the one without the protection
        select when every lane's smallest |den| (in T[1]) is at least 1e-6."""
        prot = lab(name)
        a(f"  v_cmp_ge_f32_e64 vcc, {T[1]}, {sr('TINY')}")
        a(f"  s_andn2_b64 {sp('A0')}, exec, vcc")
        a(f"  s_cbranch_scc1 {prot}")
        for k in range(K):
            short_div(dsts[k], nums[k], dens[k], protect=False)
        tail()
        a(f"{prot}:")
        for k in range(K):
            short_div(dsts[k], nums[k], dens[k])

    lab = lambda name: f".Lgp{'d' if direct else ''}{K}_{S}_{name}_%="
    # ---------------------------------------------------------- entry
    a(f"  s_mov_b32 {sr('TINY')}, {TINY:#x}")
    for k in range(K):
        a(f"  global_load_dword {xv(k)}, %[voff], %[inb] offset:{256 * k}")
    a(f"  s_getpc_b64 {sp('TB0')}")
    a(f"{lab('pc')}:")
    a(f"  s_add_u32 {sr('TB0')}, {sr('TB0')}, {lab('tbl')}-{lab('pc')}")
    a(f"  s_addc_u32 {sr('TB1')}, {sr('TB1')}, 0")
    a(f"  s_mov_b32 {sr('OFF')}, 0")
    a(f"  s_load_dword {sr('NXT')}, %[code], {sr('OFF')}")
    # one word of each of the chunk's first 256 code lines (offsets clamped to
    # the last word): the scalar loads of the words then find them in L2
    for i in range(4):
        a(f"  global_load_dword v{V_CP}, %[vc{i}], %[code]")
    a("  s_waitcnt vmcnt(0)")
    xm = lambda k: sp(f"XM{k}")
    yv = lambda k: f"v{V_Y + k}"
    for k in range(K):
        a(f"  v_cmp_lt_f32_e64 {xm(k)}, |{xv(k)}|, {sr('TINY')}")
    for k in range(K):
        op(3, f"v{V_Q + k}", xv(k), xv(k), mask=xm(k))
    # refined reciprocal of x (the division sequence's rcp and first Newton
    # step, with div_scale's identity case): used by the short stack / x
    for k in range(K):
        a(f"  v_rcp_f32_e32 {yv(k)}, {xv(k)}")
    for k in range(K):
        a(f"  v_fma_f32 {T[0]}, -{xv(k)}, {yv(k)}, 1.0")
        a(f"  v_fmac_f32_e32 {yv(k)}, {T[0]}, {yv(k)}")
    a(f"  s_mov_b32 {sr('LOSX')}, {P2(-90):#x}")
    a(f"  s_mov_b32 {sr('HISX')}, {P2(70):#x}")
    a(f"  s_mov_b32 {sr('HIXS')}, {P2(64):#x}")
    # FLG bit 0: every lane has |x| <= 2^20; bit 1: every lane has x in [2^-60, 2^60]
    a(f"  s_mov_b32 {sr('T0')}, {P2(20):#x}")
    a("  s_mov_b64 vcc, exec")
    for k in range(0, K, 2):
        a(f"  v_cmp_le_f32_e64 {sp('P0')}, |{xv(k)}|, {sr('T0')}")
        a(f"  v_cmp_le_f32_e64 {sp('J0')}, |{xv(k + 1)}|, {sr('T0')}")
        a(f"  s_and_b64 vcc, vcc, {sp('P0')}")
        a(f"  s_and_b64 vcc, vcc, {sp('J0')}")
    a(f"  s_andn2_b64 {sp('A0')}, exec, vcc")
    a(f"  s_cselect_b32 {sr('FLG')}, 0, 1")
    a(f"  s_mov_b32 {sr('T0')}, {P2(-60):#x}")
    a(f"  s_mov_b32 {sr('T1')}, {P2(60):#x}")
    a("  s_mov_b64 vcc, exec")
    for k in range(K):
        a(f"  v_cmp_ge_f32_e64 {sp('P0')}, |{xv(k)}|, {sr('T0')}")
        a(f"  v_cmp_le_f32_e64 {sp('J0')}, |{xv(k)}|, {sr('T1')}")
        a(f"  s_and_b64 vcc, vcc, {sp('P0')}")
        a(f"  s_and_b64 vcc, vcc, {sp('J0')}")
    a(f"  s_andn2_b64 {sp('A0')}, exec, vcc")
    a(f"  s_cselect_b32 {sr('T0')}, 0, 2")
    a(f"  s_or_b32 {sr('FLG')}, {sr('FLG')}, {sr('T0')}")
    # FLG bit 2: no lane has |x| < 1e-6, so dividing by x needs no protection select
    reduce_abs("min", T[0], [xv(k) for k in range(K)])
    a(f"  v_cmp_ge_f32_e64 vcc, {T[0]}, {sr('TINY')}")
    a(f"  s_andn2_b64 {sp('A0')}, exec, vcc")
    a(f"  s_cselect_b32 {sr('T0')}, 0, 4")
    a(f"  s_or_b32 {sr('FLG')}, {sr('FLG')}, {sr('T0')}")
    tail()
    # ---------------------------------------------------------- table
    handlers = {}
    for key in range(1024):
        f, mode, d = key & 3, (key >> 2) & 7, key >> 5
        name = None
        if key == END_KEY:
            name = "end"
        elif d < S and mode in (M_XX, M_XS, M_SX):
            name = f"h{key}"
        elif d + 1 < S and mode in (M_SS, M_RS):
            name = f"h{key}"
        elif d < S and f == 0 and mode in (M_PUSH, M_LOAD, M_STORE):
            name = f"h{key}"
        else:
            name = "end"          # never emitted by the compiler; ends the chunk
        handlers[key] = name
    # ---------------------------------------------------------- handlers
    def emit(key):
        f, mode, d = key & 3, (key >> 2) & 7, key >> 5
        if mode == M_XX and f == 3:
            for k in range(K):
                a(f"  v_mov_b32_e32 {st(d, k)}, v{V_Q + k}")
        elif mode == M_XX:
            for k in range(K):
                op(f, st(d, k), xv(k), xv(k))
        elif mode == M_XS and f == 3:
            slow = lab(f"xs{d}")
            a(f"  s_bitcmp0_b32 {sr('FLG')}, 1")
            a(f"  s_cbranch_scc1 {slow}")
            reduce_abs("max", T[2], [st(d, k) for k in range(K)])
            a(f"  v_cmp_le_f32_e64 vcc, {T[2]}, {sr('HIXS')}")
            a(f"  s_andn2_b64 {sp('A0')}, exec, vcc")
            a(f"  s_cbranch_scc1 {slow}")
            reduce_abs("min", T[1], [st(d, k) for k in range(K)])
            short_div_both(f"xsp{d}", [st(d, k) for k in range(K)], [xv(k) for k in range(K)],
                           [st(d, k) for k in range(K)])
            tail()
            a(f"{slow}:")
            for k in range(K):
                op(f, st(d, k), xv(k), st(d, k))
        elif mode == M_XS:
            for k in range(K):
                op(f, st(d, k), xv(k), st(d, k))
        elif mode == M_SX and f == 3:
            slow = lab(f"sx{d}")
            a(f"  s_bitcmp0_b32 {sr('FLG')}, 0")
            a(f"  s_cbranch_scc1 {slow}")
            reduce_abs("min", T[1], [st(d, k) for k in range(K)])
            reduce_abs("max", T[2], [st(d, k) for k in range(K)])
            a(f"  v_cmp_ge_f32_e64 {sp('P0')}, {T[1]}, {sr('LOSX')}")
            a(f"  v_cmp_le_f32_e64 vcc, {T[2]}, {sr('HISX')}")
            a(f"  s_and_b64 vcc, vcc, {sp('P0')}")
            a(f"  s_andn2_b64 {sp('A0')}, exec, vcc")
            a(f"  s_cbranch_scc1 {slow}")
            unprot = lab(f"sxu{d}")
            a(f"  s_bitcmp1_b32 {sr('FLG')}, 2")
            a(f"  s_cbranch_scc1 {unprot}")
            for protect in (True, False):
                if not protect:
                    a(f"{unprot}:")
                for k in range(K):
                    n, x, y = st(d, k), xv(k), yv(k)
                    a(f"  v_mul_f32_e32 {T[3]}, {n}, {y}")
                    a(f"  v_fma_f32 {T[4]}, -{x}, {T[3]}, {n}")
                    if protect:
                        a(f"  v_fma_f32 {T[0]}, {T[4]}, {y}, {T[3]}")
                        a(f"  v_cndmask_b32_e64 {n}, {T[0]}, 1.0, {xm(k)}")
                    else:
                        a(f"  v_fma_f32 {n}, {T[4]}, {y}, {T[3]}")
                tail()
            a(f"{slow}:")
            for k in range(K):
                op(f, st(d, k), st(d, k), xv(k), mask=xm(k))
        elif mode == M_SX:
            for k in range(K):
                op(f, st(d, k), st(d, k), xv(k), mask=xm(k))
        elif mode in (M_SS, M_RS) and f == 3:
            # stack / stack: the x / stack conditions with the numerator's
            # range checked per case: |num| in [2^-60, 2^60], |den| <= 2^64
            slow = lab(f"ss{mode}_{d}")
            num = [st(d, k) if mode == M_SS else st(d + 1, k) for k in range(K)]
            den = [st(d + 1, k) if mode == M_SS else st(d, k) for k in range(K)]
            reduce_abs("max", T[0], num)
            reduce_abs("min", T[1], num)
            reduce_abs("max", T[2], den)
            a(f"  v_cmp_ge_f32_e32 vcc, {P2(60):#x}, {T[0]}")
            a(f"  s_mov_b64 {sp('P0')}, vcc")
            a(f"  v_cmp_le_f32_e32 vcc, {P2(-60):#x}, {T[1]}")
            a(f"  s_and_b64 {sp('P0')}, {sp('P0')}, vcc")
            a(f"  v_cmp_le_f32_e64 vcc, {T[2]}, {sr('HIXS')}")
            a(f"  s_and_b64 vcc, vcc, {sp('P0')}")
            a(f"  s_andn2_b64 {sp('A0')}, exec, vcc")
            a(f"  s_cbranch_scc1 {slow}")
            reduce_abs("min", T[1], den)
            short_div_both(f"ssp{mode}_{d}", [st(d, k) for k in range(K)], num, den)
            tail()
            a(f"{slow}:")
            for k in range(K):
                op(f, st(d, k), num[k], den[k])
        elif mode == M_SS:
            for k in range(K):
                op(f, st(d, k), st(d, k), st(d + 1, k))
        elif mode == M_RS:
            for k in range(K):
                op(f, st(d, k), st(d + 1, k), st(d, k))
        elif mode == M_PUSH:
            a(f"  s_lshr_b32 {sr('T0')}, {sr('INS')}, 10")
            a(f"  s_cmp_eq_u32 {sr('T0')}, 0")
            a(f"  s_cbranch_scc1 {lab(f'px{d}')}")
            a(f"  s_mul_i32 {sr('T0')}, {sr('T0')}, %[strideb]")
            a(f"  s_add_u32 {sr('A0')}, %[inb_lo], {sr('T0')}")
            a(f"  s_addc_u32 {sr('A1')}, %[inb_hi], 0")
            for k in range(K):
                a(f"  global_load_dword {st(d, k)}, %[voff], {sp('A0')} offset:{256 * k}")
            a("  s_waitcnt vmcnt(0)")
            tail()
            a(f"{lab(f'px{d}')}:")
            for k in range(K):
                a(f"  v_mov_b32_e32 {st(d, k)}, {xv(k)}")
        elif mode == M_LOAD:
            a(f"  s_lshr_b32 {sr('T0')}, {sr('INS')}, 10")
            a(f"  s_lshl_b32 {sr('T0')}, {sr('T0')}, 2")
            a(f"  s_load_dword {sr('T1')}, %[cin], {sr('T0')}")
            a("  s_waitcnt lgkmcnt(0)")
            a(f"  s_mul_i32 {sr('A0')}, {sr('T1')}, %[strideb]")
            a(f"  s_mul_hi_u32 {sr('A1')}, {sr('T1')}, %[strideb]")
            a(f"  s_add_u32 {sr('A0')}, {sr('A0')}, %[vb_lo]")
            a(f"  s_addc_u32 {sr('A1')}, {sr('A1')}, %[vb_hi]")
            for k in range(K):
                a(f"  global_load_dword {st(d, k)}, %[voff], {sp('A0')} offset:{256 * k}{SHARED}")
            a("  s_waitcnt vmcnt(0)")
        elif mode == M_STORE:
            a(f"  s_lshr_b32 {sr('T0')}, {sr('INS')}, 10")
            a(f"  s_mul_i32 {sr('A0')}, {sr('T0')}, %[strideb]")
            a(f"  s_mul_hi_u32 {sr('A1')}, {sr('T0')}, %[strideb]")
            a(f"  s_add_u32 {sr('A0')}, {sr('A0')}, %[rb_lo]")
            a(f"  s_addc_u32 {sr('A1')}, {sr('A1')}, %[rb_hi]")
            for k in range(K):
                a(f"  global_store_dword %[voff], {st(d, k)}, {sp('A0')} offset:{256 * k}")
        tail()

    def in_slot(key):
        """+, -, x (and the copy of x / x): the handler and the next word's
        dispatch fit the key's slot.  Divides, PUSH, LOAD and STORE are out of
        line, one branch away."""
        f, mode = key & 3, (key >> 2) & 7
        return handlers[key] == f"h{key}" and (mode == M_XX or (f != 3 and mode in (M_XS, M_SX, M_SS, M_RS)))

    if not direct:
        a(f"{lab('tbl')}:")
        for key in range(1024):
            a(f"  s_branch {lab(handlers[key])}")
        for key in range(1024):
            if handlers[key] == f"h{key}":
                a(f"{lab(handlers[key])}:")
                emit(key)
        a(f"{lab('end')}:")
    # out-of-line handlers and the way out, before the slots (within a branch's reach)
    for key in range(1024 if direct else 0):
        if handlers[key] == f"h{key}" and not in_slot(key):
            assert key * SLOT < 64 * 1024
            a(f"{lab(handlers[key])}:")
            emit(key)
    if direct:
        a(f"{lab('endjump')}:")
        a(f"  s_add_u32 {sr('TG0')}, {sr('TB0')}, {1024 * SLOT:#x}")
        a(f"  s_addc_u32 {sr('TG1')}, {sr('TB1')}, 0")
        a(f"  s_setpc_b64 {sp('TG0')}")
        # ------------------------------------------------------ slots
        a(f"  .p2align {SLOT.bit_length() - 1}")
        a(f"{lab('tbl')}:")
    for key in range(1024 if direct else 0):
        slot = lab(f"s{key}")
        if key:
            a(f"  .p2align {SLOT.bit_length() - 1}")
        a(f"{slot}:")
        if in_slot(key):
            emit(key)
        elif handlers[key] == f"h{key}":
            a(f"  s_branch {lab(handlers[key])}")
        else:
            a(f"  s_branch {lab('endjump') if key < 512 else lab('end')}")
        a(f"  .if . - {slot} > {SLOT}")
        a(f"  .error \"dispatch slot {key} is longer than {SLOT} bytes\"")
        a("  .endif")
    if direct:              # the end, at table + 1024 * SLOT
        a(f"  .p2align {SLOT.bit_length() - 1}")
        a(f"{lab('end')}:")
    a("  s_waitcnt lgkmcnt(0)")
    for k in range(K):
        a(f"  global_store_dword %[voff], {st(0, k)}, %[outb] offset:{256 * k}{SHARED}")
    a("  s_waitcnt vmcnt(0)")

    body = "\n".join('        "' + line.replace('"', '\\"') + '\\n"' for line in L)
    vclob = ", ".join(f'"v{i}"' for i in range(V_ST, n_vgpr))
    sclob = ", ".join(f'"s{s[n]}"' for n in names)
    return f"""
// K = {K} cases per lane, S = {S} stack slots: v{V_ST}..v{n_vgpr - 1}, s{S_BASE}..s{S_BASE + len(names) - 1}.
__device__ __forceinline__ void run_f32{'d' if direct else ''}_dispatch_{K}_{S}(const GP_CONST uint32_t* code, const float* inb,
                                                     const float* vb, float* rb, const GP_CONST int32_t* cin,
                                                     uint32_t strideb, float* outb, uint32_t voff,
                                                     uint32_t vc0, uint32_t vc1, uint32_t vc2, uint32_t vc3)
{{
    const uint64_t inb64 = (uint64_t)inb, vb64 = (uint64_t)vb, rb64 = (uint64_t)rb;
    asm volatile(
{body}
        :
        : [code] "s"(code), [inb] "s"(inb), [inb_lo] "s"((uint32_t)inb64), [inb_hi] "s"((uint32_t)(inb64 >> 32)),
          [vb_lo] "s"((uint32_t)vb64), [vb_hi] "s"((uint32_t)(vb64 >> 32)),
          [rb_lo] "s"((uint32_t)rb64), [rb_hi] "s"((uint32_t)(rb64 >> 32)), [cin] "s"(cin),
          [strideb] "s"(strideb), [outb] "s"(outb), [voff] "v"(voff),
          [vc0] "v"(vc0), [vc1] "v"(vc1), [vc2] "v"(vc2), [vc3] "v"(vc3)
        : "memory", "vcc", "scc", {sclob},
          {vclob});
}}
"""


# ---------------------------------------------------------------- Boolean
# The Boolean loop (dispatch_bool.inc): K 64-bit words (64 cases each) per
# lane, a value being a VGPR pair (lo, hi).  The input words of the slice,
# up to NI inputs, are loaded into VGPRs when the chunk starts; an instruction
# names an input by its payload, a wave-uniform index, so the handler reads it
# in GPR index mode (register number offset by an SGPR) rather than from LDS.
# The vectors of the chunk's first BOOL_NP LOAD inputs are fetched together
# with the input words when the chunk starts (a chunk runs only once all its
# inputs are done), so that a LOAD costs register moves instead of a memory
# round trip on the chains of chunks that bound this launch.
BOOL_VARIANTS = [(1, 10), (2, 10)]
BOOL_NI = 16
BOOL_NP = 4


def gen_bool(K: int, S: int, NI: int = BOOL_NI, NP: int = BOOL_NP) -> str:
    V_IN = V_ST + S * K * 2
    V_T = V_IN + NI * K * 2
    V_PF = V_T + 4 * K
    n_vgpr = V_PF + NP * K * 2
    names = []
    for p in ["TB", "TG", "A"]:
        names += [f"{p}0", f"{p}1"]
    names += ["INS", "NXT", "OFF", "T0", "T1", "J"] + [f"P{j}" for j in range(NP)]
    s = {n: S_BASE + i for i, n in enumerate(names)}
    sr = lambda n: f"s{s[n]}"
    sp = lambda n: f"s[{s[n]}:{s[n] + 1}]"
    st = lambda d, k, h: f"v{V_ST + (d * K + k) * 2 + h}"
    inp = lambda k, h: f"v{V_IN + k * 2 + h}"          # input 0; M0 moves to input j
    ta = lambda k, h: f"v{V_T + k * 2 + h}"             # first operand read from the inputs
    tb = lambda k, h: f"v{V_T + 2 * K + k * 2 + h}"     # second
    L = []
    a = L.append
    lab = lambda name: f".Lgb{K}_{S}_{name}_%="

    def tail():
        a("  s_waitcnt lgkmcnt(0)")
        a(f"  s_mov_b32 {sr('INS')}, {sr('NXT')}")
        a(f"  s_add_u32 {sr('OFF')}, {sr('OFF')}, 4")
        a(f"  s_load_dword {sr('NXT')}, %[code], {sr('OFF')}")
        a(f"  s_and_b32 {sr('TG0')}, {sr('INS')}, 0x3ff")
        a(f"  s_lshl2_add_u32 {sr('TG0')}, {sr('TG0')}, {sr('TB0')}")
        a(f"  s_addc_u32 {sr('TG1')}, {sr('TB1')}, 0")
        a(f"  s_setpc_b64 {sp('TG0')}")

    def read_input(idx_sreg, dst, base=V_IN):
        """dst(k, h) = row idx, word k, half h of the rows held from register
        base on, read idx * 2K registers past the first row in GPR index mode
        (the offset applies to SRC0 of the moves in between)."""
        a(f"  s_lshl_b32 {sr('J')}, {idx_sreg}, {(2 * K).bit_length() - 1}")
        a(f"  s_set_gpr_idx_on {sr('J')}, gpr_idx(SRC0)")
        for k in range(K):
            for h in range(2):
                a(f"  v_mov_b32_e32 {dst(k, h)}, v{base + k * 2 + h}")
        a("  s_set_gpr_idx_off")

    def op64(f, d, k, A, B):
        for h in range(2):
            dst = st(d, k, h)
            a(f"  v_{'and' if f in (0, 2) else 'or'}_b32_e32 {dst}, {A(k, h)}, {B(k, h)}")
            if f >= 2:
                a(f"  v_not_b32_e32 {dst}, {dst}")

    # ---------------------------------------------------------- entry
    a(f"  s_getpc_b64 {sp('TB0')}")
    a(f"{lab('pc')}:")
    a(f"  s_add_u32 {sr('TB0')}, {sr('TB0')}, {lab('tbl')}-{lab('pc')}")
    a(f"  s_addc_u32 {sr('TB1')}, {sr('TB1')}, 0")
    a(f"  s_mov_b32 {sr('OFF')}, 0")
    a(f"  s_load_dword {sr('NXT')}, %[code], {sr('OFF')}")
    # one word of each of the chunk's first 64 code lines (64 bytes apart; the
    # offset is clamped to the last word), so that the scalar loads of the
    # words find their lines in L2
    a(f"  global_load_dword {ta(0, 0)}, %[vcoff], %[code]")
    # the vectors of LOAD inputs 0 .. min(nload, NP) - 1: their slots, then the rows
    a("  s_cmp_eq_u32 %[nload], 0")
    a(f"  s_cbranch_scc1 {lab('pfok')}")
    for j in range(NP):
        if j:
            a(f"  s_cmp_le_u32 %[nload], {j}")
            a(f"  s_cbranch_scc1 {lab('pfslots')}")
        a(f"  s_load_dword {sr(f'P{j}')}, %[cin], {4 * j}")
    a(f"{lab('pfslots')}:")
    a("  s_waitcnt lgkmcnt(0)")
    for j in range(NP):
        if j:
            a(f"  s_cmp_le_u32 %[nload], {j}")
            a(f"  s_cbranch_scc1 {lab('pfok')}")
        a(f"  s_mul_i32 {sr('A0')}, {sr(f'P{j}')}, %[strideb]")
        a(f"  s_mul_hi_u32 {sr('A1')}, {sr(f'P{j}')}, %[strideb]")
        a(f"  s_add_u32 {sr('A0')}, {sr('A0')}, %[vb_lo]")
        a(f"  s_addc_u32 {sr('A1')}, {sr('A1')}, %[vb_hi]")
        for k in range(K):
            a(f"  global_load_dwordx2 v[{V_PF + (j * K + k) * 2}:{V_PF + (j * K + k) * 2 + 1}], %[voff], "
              f"{sp('A0')} offset:{512 * k}{SHARED}")
    a(f"{lab('pfok')}:")
    # the slice's input words: row j at inb + j * strideb, for j < n_inputs
    a(f"  s_mov_b32 {sr('A0')}, %[inb_lo]")
    a(f"  s_mov_b32 {sr('A1')}, %[inb_hi]")
    for j in range(NI):
        a(f"  s_cmp_le_u32 %[nin], {j}")
        a(f"  s_cbranch_scc1 {lab('inok')}")
        for k in range(K):
            a(f"  global_load_dwordx2 v[{V_IN + (j * K + k) * 2}:{V_IN + (j * K + k) * 2 + 1}], %[voff], "
              f"{sp('A0')} offset:{512 * k}")
        a(f"  s_add_u32 {sr('A0')}, {sr('A0')}, %[strideb]")
        a(f"  s_addc_u32 {sr('A1')}, {sr('A1')}, 0")
    a(f"{lab('inok')}:")
    a("  s_waitcnt vmcnt(0)")
    tail()
    # ---------------------------------------------------------- table
    handlers = {}
    for key in range(1024):
        f, mode, d = key & 3, (key >> 2) & 7, key >> 5
        if key == END_KEY:
            handlers[key] = "end"
        elif d < S and mode in (M_XX, M_XS):
            handlers[key] = f"h{key}"
        elif d + 1 < S and mode == M_SS:
            handlers[key] = f"h{key}"
        elif d < S and f == 0 and mode in (M_PUSH, M_LOAD, M_STORE):
            handlers[key] = f"h{key}"
        else:
            handlers[key] = "end"     # never emitted for Boolean programs; ends the chunk
    a(f"{lab('tbl')}:")
    for key in range(1024):
        a(f"  s_branch {lab(handlers[key])}")
    # ---------------------------------------------------------- handlers
    for key in range(1024):
        if handlers[key] != f"h{key}":
            continue
        f, mode, d = key & 3, (key >> 2) & 7, key >> 5
        a(f"{lab(handlers[key])}:")
        if mode == M_XX:                 # f(input a, input b), a = payload & 2047, b = payload >> 11
            a(f"  s_lshr_b32 {sr('T0')}, {sr('INS')}, 10")
            a(f"  s_and_b32 {sr('T1')}, {sr('T0')}, 0x7ff")
            a(f"  s_lshr_b32 {sr('T0')}, {sr('T0')}, 11")
            read_input(sr('T1'), ta)
            read_input(sr('T0'), tb)
            for k in range(K):
                op64(f, d, k, ta, tb)
        elif mode == M_XS:               # f(input payload, slot d)
            a(f"  s_lshr_b32 {sr('T0')}, {sr('INS')}, 10")
            read_input(sr('T0'), ta)
            for k in range(K):
                op64(f, d, k, ta, lambda k_, h: st(d, k_, h))
        elif mode == M_SS:
            for k in range(K):
                op64(f, d, k, lambda k_, h: st(d, k_, h), lambda k_, h: st(d + 1, k_, h))
        elif mode == M_PUSH:
            a(f"  s_lshr_b32 {sr('T0')}, {sr('INS')}, 10")
            read_input(sr('T0'), lambda k, h: st(d, k, h))
        elif mode == M_LOAD:
            a(f"  s_lshr_b32 {sr('T0')}, {sr('INS')}, 10")
            a(f"  s_cmp_lt_u32 {sr('T0')}, {NP}")
            a(f"  s_cbranch_scc0 {lab(f'ld{key}')}")
            read_input(sr('T0'), lambda k, h: st(d, k, h), V_PF)     # fetched when the chunk started
            tail()
            a(f"{lab(f'ld{key}')}:")
            a(f"  s_lshl_b32 {sr('T0')}, {sr('T0')}, 2")
            a(f"  s_load_dword {sr('T1')}, %[cin], {sr('T0')}")
            a("  s_waitcnt lgkmcnt(0)")
            a(f"  s_mul_i32 {sr('A0')}, {sr('T1')}, %[strideb]")
            a(f"  s_mul_hi_u32 {sr('A1')}, {sr('T1')}, %[strideb]")
            a(f"  s_add_u32 {sr('A0')}, {sr('A0')}, %[vb_lo]")
            a(f"  s_addc_u32 {sr('A1')}, {sr('A1')}, %[vb_hi]")
            for k in range(K):
                a(f"  global_load_dwordx2 v[{V_ST + (d * K + k) * 2}:{V_ST + (d * K + k) * 2 + 1}], %[voff], "
                  f"{sp('A0')} offset:{512 * k}{SHARED}")
            a("  s_waitcnt vmcnt(0)")
        elif mode == M_STORE:
            a(f"  s_lshr_b32 {sr('T0')}, {sr('INS')}, 10")
            a(f"  s_mul_i32 {sr('A0')}, {sr('T0')}, %[strideb]")
            a(f"  s_mul_hi_u32 {sr('A1')}, {sr('T0')}, %[strideb]")
            a(f"  s_add_u32 {sr('A0')}, {sr('A0')}, %[rb_lo]")
            a(f"  s_addc_u32 {sr('A1')}, {sr('A1')}, %[rb_hi]")
            for k in range(K):
                a(f"  global_store_dwordx2 %[voff], v[{V_ST + (d * K + k) * 2}:{V_ST + (d * K + k) * 2 + 1}], "
                  f"{sp('A0')} offset:{512 * k}")
        tail()
    # ---------------------------------------------------------- end
    a(f"{lab('end')}:")
    a("  s_waitcnt lgkmcnt(0)")
    for k in range(K):
        a(f"  global_store_dwordx2 %[voff], v[{V_ST + k * 2}:{V_ST + k * 2 + 1}], %[outb] offset:{512 * k}{SHARED}")
    a("  s_waitcnt vmcnt(0)")

    body = "\n".join(f'        "{line}\\n"' for line in L)
    vclob = ", ".join(f'"v{i}"' for i in range(V_ST, n_vgpr))
    sclob = ", ".join(f'"s{s[n]}"' for n in names)
    return f"""
// K = {K} words per lane, S = {S} stack slots, up to {NI} inputs, {NP} LOAD inputs fetched ahead:
// v{V_ST}..v{n_vgpr - 1}, s{S_BASE}..s{S_BASE + len(names) - 1}.
__device__ __forceinline__ void run_bool_dispatch_{K}_{S}(const GP_CONST uint32_t* code, const uint64_t* inb,
                                                      const uint64_t* vb, uint64_t* rb, const GP_CONST int32_t* cin,
                                                      uint32_t strideb, uint64_t* outb, uint32_t voff, uint32_t nin,
                                                      uint32_t nload, uint32_t vcoff)
{{
    const uint64_t inb64 = (uint64_t)inb, vb64 = (uint64_t)vb, rb64 = (uint64_t)rb;
    asm volatile(
{body}
        :
        : [code] "s"(code), [inb_lo] "s"((uint32_t)inb64), [inb_hi] "s"((uint32_t)(inb64 >> 32)),
          [vb_lo] "s"((uint32_t)vb64), [vb_hi] "s"((uint32_t)(vb64 >> 32)),
          [rb_lo] "s"((uint32_t)rb64), [rb_hi] "s"((uint32_t)(rb64 >> 32)), [cin] "s"(cin),
          [strideb] "s"(strideb), [outb] "s"(outb), [voff] "v"(voff), [nin] "s"(nin), [nload] "s"(nload),
          [vcoff] "v"(vcoff)
        : "memory", "vcc", "scc", "m0", {sclob},
          {vclob});
}}
"""


# ---------------------------------------------------------- one Boolean word
# When every test case fits in one 64-bit word (T <= 64) a chunk's value is
# the same for the whole wave, so this loop keeps it on the scalar unit: the
# stack slots st[d] and the input words in[j] are SGPR pairs, the handlers
# use the scalar unit's 64-bit AND, OR, NAND and NOR, and a handler picks
# input j by relative SGPR addressing (s_movrels_b64 with M0 = 2j, one wait
# state after M0 is written).  Vector memory is used only where other waves
# are involved: LOAD reads lane 0's word of a chunk vector with an
# agent-coherent vector load, and STORE and the chunk's end write lane 0's
# word (every other lane is masked off for those loads and stores).
#
# Dispatch is direct: the handler of key k (with the fetch of the next-but-one
# word and the jump to the next word's handler) fills a slot of BOOLW_SLOT
# bytes at table + k * BOOLW_SLOT, so a word costs one jump instead of the
# table's two (the slot's start is computed, not read).  The assembler checks
# that no slot outgrows its place; code that would (the LOADs past the ones
# fetched ahead) and the way out sit before the slots, within a branch's reach.
BOOLW_S = 10
BOOLW_NI = 8
BOOLW_NP = 4
BOOLW_SBASE = 40
BOOLW_SLOT = 128


def gen_bool_word(S: int = BOOLW_S, NI: int = BOOLW_NI, NP: int = BOOLW_NP, SLOT: int = BOOLW_SLOT) -> str:
    assert SLOT & (SLOT - 1) == 0 and S <= 16       # the key's top bit is then 0 (see the handlers)
    names = []
    for p in ["TB", "TG", "X", "Y"] + [f"ST{d}" for d in range(S)] + [f"IN{j}" for j in range(NI)] + \
            [f"LD{j}" for j in range(NP)]:
        names += [f"{p}0", f"{p}1"]                   # pairs first: all even-aligned
    names += ["INS", "NXT", "OFF", "T0", "T1"]
    s = {n: BOOLW_SBASE + i for i, n in enumerate(names)}
    assert BOOLW_SBASE % 2 == 0 and BOOLW_SBASE + len(names) <= 100
    sr = lambda n: f"s{s[n]}"
    sp = lambda n: f"s[{s[n + '0']}:{s[n + '0'] + 1}]"
    V_CP, V_T, V_PF = 16, 18, 20                      # code-line touches, a word, the prefetched LOAD words
    n_vgpr = V_PF + 2 * NP
    OPS = ["s_and_b64", "s_or_b64", "s_nand_b64", "s_nor_b64"]
    L = []
    a = L.append
    lab = lambda name: f".Lgw{S}_{name}_%="

    def tail(advanced=False):
        # the handler of key k starts at table + k * SLOT: one jump per word.
        # advanced: the handler has already stepped OFF (in the wait state an
        # s_movrels needs after M0 is written)
        a("  s_waitcnt lgkmcnt(0)")
        a(f"  s_mov_b32 {sr('INS')}, {sr('NXT')}")
        if not advanced:
            a(f"  s_add_u32 {sr('OFF')}, {sr('OFF')}, 4")
        a(f"  s_load_dword {sr('NXT')}, %[code], {sr('OFF')}")
        a(f"  s_and_b32 {sr('TG0')}, {sr('INS')}, 0x3ff")
        a(f"  s_lshl_b32 {sr('TG0')}, {sr('TG0')}, {SLOT.bit_length() - 1}")
        a(f"  s_add_u32 {sr('TG0')}, {sr('TG0')}, {sr('TB0')}")
        a(f"  s_addc_u32 {sr('TG1')}, {sr('TB1')}, 0")
        a(f"  s_setpc_b64 {sp('TG')}")

    def lane0_store(src, addr, shared):
        """Lane 0 writes the SGPR pair src to the 8 bytes at addr + voff."""
        a(f"  s_mov_b64 {sp('Y')}, exec")
        a("  s_mov_b64 exec, 1")
        a(f"  v_mov_b32_e32 v{V_T}, {sr(src + '0')}")
        a(f"  v_mov_b32_e32 v{V_T + 1}, {sr(src + '1')}")
        a(f"  global_store_dwordx2 %[voff], v[{V_T}:{V_T + 1}], {addr}{shared}")
        a(f"  s_mov_b64 exec, {sp('Y')}")

    def row_address(slot_sreg, lo, hi):
        a(f"  s_mul_i32 {sr('X0')}, {slot_sreg}, %[strideb]")
        a(f"  s_mul_hi_u32 {sr('X1')}, {slot_sreg}, %[strideb]")
        a(f"  s_add_u32 {sr('X0')}, {sr('X0')}, {lo}")
        a(f"  s_addc_u32 {sr('X1')}, {sr('X1')}, {hi}")

    # ---------------------------------------------------------- entry
    a(f"  s_getpc_b64 {sp('TB')}")
    a(f"{lab('pc')}:")
    a(f"  s_add_u32 {sr('TB0')}, {sr('TB0')}, {lab('tbl')}-{lab('pc')}")
    a(f"  s_addc_u32 {sr('TB1')}, {sr('TB1')}, 0")
    a(f"  s_mov_b32 {sr('OFF')}, 0")
    a(f"  s_load_dword {sr('NXT')}, %[code], {sr('OFF')}")
    # one word of each of the chunk's first 64 code lines (offset clamped to
    # the last word), so that the scalar loads of the words find them in L2;
    # nothing reads v{V_CP}, and the chunk's end waits for the load
    a(f"  global_load_dword v{V_CP}, %[vcoff], %[code]")
    # the vector slots of LOAD inputs 0 .. min(nload, NP) - 1 (into LD{j}0)
    a("  s_cmp_eq_u32 %[nload], 0")
    a(f"  s_cbranch_scc1 {lab('slots')}")
    for j in range(NP):
        if j:
            a(f"  s_cmp_le_u32 %[nload], {j}")
            a(f"  s_cbranch_scc1 {lab('slots')}")
        a(f"  s_load_dword {sr(f'LD{j}0')}, %[cin], {4 * j}")
    a(f"{lab('slots')}:")
    # the input words: row j at inb + j * strideb, for j < nin
    a(f"  s_mov_b32 {sr('T1')}, 0")
    for j in range(NI):
        a(f"  s_cmp_le_u32 %[nin], {j}")
        a(f"  s_cbranch_scc1 {lab('inok')}")
        a(f"  s_load_dwordx2 {sp(f'IN{j}')}, %[inb], {sr('T1')}")
        a(f"  s_add_u32 {sr('T1')}, {sr('T1')}, %[strideb]")
    a(f"{lab('inok')}:")
    a("  s_waitcnt lgkmcnt(0)")
    a("  s_cmp_eq_u32 %[nload], 0")
    a(f"  s_cbranch_scc1 {lab('pfok')}")
    a(f"  s_mov_b64 {sp('Y')}, exec")               # lane 0 alone reads the vectors' words
    a("  s_mov_b64 exec, 1")
    for j in range(NP):
        if j:
            a(f"  s_cmp_le_u32 %[nload], {j}")
            a(f"  s_cbranch_scc1 {lab('pfwait')}")
        row_address(sr(f'LD{j}0'), "%[vb_lo]", "%[vb_hi]")
        a(f"  global_load_dwordx2 v[{V_PF + 2 * j}:{V_PF + 2 * j + 1}], %[voff], {sp('X')}{SHARED}")
    a(f"{lab('pfwait')}:")
    a(f"  s_mov_b64 exec, {sp('Y')}")
    a("  s_waitcnt vmcnt(0)")
    for j in range(NP):              # lane 0's word; pairs past nload are never read
        a(f"  v_readfirstlane_b32 {sr(f'LD{j}0')}, v{V_PF + 2 * j}")
        a(f"  v_readfirstlane_b32 {sr(f'LD{j}1')}, v{V_PF + 2 * j + 1}")
    a(f"{lab('pfok')}:")
    tail()
    # ---------------------------------------------------------- slots
    handlers = {}
    for key in range(1024):
        f, mode, d = key & 3, (key >> 2) & 7, key >> 5
        if key == END_KEY:
            handlers[key] = False
        elif d < S and mode in (M_XX, M_XS):
            handlers[key] = True
        elif d + 1 < S and mode == M_SS:
            handlers[key] = True
        elif d < S and f == 0 and mode in (M_PUSH, M_LOAD, M_STORE):
            handlers[key] = True
        else:
            handlers[key] = False     # never emitted for Boolean programs; ends the chunk
    # Out-of-line code, before the slots so that branches to it stay within
    # the +-128 KiB a branch reaches: the LOADs past the ones fetched ahead,
    # and the jump to the chunk's end, which follows the last slot.
    for key in range(1024):
        f, mode, d = key & 3, (key >> 2) & 7, key >> 5
        if not handlers[key] or mode != M_LOAD:
            continue
        assert key * SLOT < 96 * 1024
        a(f"{lab(f'ld{key}')}:")
        a(f"  s_lshl_b32 {sr('T0')}, {sr('T0')}, 2")
        a(f"  s_load_dword {sr('T1')}, %[cin], {sr('T0')}")
        a("  s_waitcnt lgkmcnt(0)")
        row_address(sr('T1'), "%[vb_lo]", "%[vb_hi]")
        a(f"  s_mov_b64 {sp('Y')}, exec")
        a("  s_mov_b64 exec, 1")
        a(f"  global_load_dwordx2 v[{V_T}:{V_T + 1}], %[voff], {sp('X')}{SHARED}")
        a(f"  s_mov_b64 exec, {sp('Y')}")
        a("  s_waitcnt vmcnt(0)")
        a(f"  v_readfirstlane_b32 {sr(f'ST{d}0')}, v{V_T}")
        a(f"  v_readfirstlane_b32 {sr(f'ST{d}1')}, v{V_T + 1}")
        tail()
    a(f"{lab('endjump')}:")
    a(f"  s_add_u32 {sr('TG0')}, {sr('TB0')}, {1024 * SLOT:#x}")
    a(f"  s_addc_u32 {sr('TG1')}, {sr('TB1')}, 0")
    a(f"  s_setpc_b64 {sp('TG')}")
    a(f"  .p2align {SLOT.bit_length() - 1}")
    a(f"{lab('tbl')}:")
    for key in range(1024):
        f, mode, d = key & 3, (key >> 2) & 7, key >> 5
        st = f"ST{d}"
        slot = lab(f"s{key}")
        if key:
            a(f"  .p2align {SLOT.bit_length() - 1}")
        a(f"{slot}:")
        if not handlers[key]:
            a(f"  s_branch {lab('endjump') if key < 512 else lab('end')}")
        # A word is key | payload << 10 and the key's top bit is 0 (d < 16), so
        # INS >> 9 is twice the payload: M0 for the SGPR pair it names.
        elif mode == M_XX:               # f(input a, input b), a = payload & 2047, b = payload >> 11
            a(f"  s_lshr_b32 {sr('T1')}, {sr('INS')}, 9")
            a(f"  s_and_b32 m0, {sr('T1')}, 0xffe")
            a(f"  s_lshr_b32 {sr('T0')}, {sr('INS')}, 21")
            a(f"  s_movrels_b64 {sp('X')}, {sp('IN0')}")
            a(f"  s_lshl_b32 m0, {sr('T0')}, 1")
            a(f"  s_add_u32 {sr('OFF')}, {sr('OFF')}, 4")
            a(f"  s_movrels_b64 {sp('Y')}, {sp('IN0')}")
            a(f"  {OPS[f]} {sp(st)}, {sp('X')}, {sp('Y')}")
            tail(advanced=True)
        elif mode == M_XS:               # f(input payload, slot d)
            a(f"  s_lshr_b32 m0, {sr('INS')}, 9")
            a(f"  s_add_u32 {sr('OFF')}, {sr('OFF')}, 4")
            a(f"  s_movrels_b64 {sp('X')}, {sp('IN0')}")
            a(f"  {OPS[f]} {sp(st)}, {sp('X')}, {sp(st)}")
            tail(advanced=True)
        elif mode == M_SS:
            a(f"  {OPS[f]} {sp(st)}, {sp(st)}, {sp(f'ST{d + 1}')}")
            tail()
        elif mode == M_PUSH:
            a(f"  s_lshr_b32 m0, {sr('INS')}, 9")
            a(f"  s_add_u32 {sr('OFF')}, {sr('OFF')}, 4")
            a(f"  s_movrels_b64 {sp(st)}, {sp('IN0')}")
            tail(advanced=True)
        elif mode == M_LOAD:
            a(f"  s_lshr_b32 {sr('T0')}, {sr('INS')}, 10")
            a(f"  s_cmp_lt_u32 {sr('T0')}, {NP}")
            a(f"  s_cbranch_scc0 {lab(f'ld{key}')}")
            a(f"  s_lshr_b32 m0, {sr('INS')}, 9")         # fetched when the chunk started
            a(f"  s_add_u32 {sr('OFF')}, {sr('OFF')}, 4")
            a(f"  s_movrels_b64 {sp(st)}, {sp('LD0')}")
            tail(advanced=True)
        elif mode == M_STORE:
            a(f"  s_lshr_b32 {sr('T0')}, {sr('INS')}, 10")
            row_address(sr('T0'), "%[rb_lo]", "%[rb_hi]")
            lane0_store(st, sp('X'), "")
            tail()
        # the assembler refuses a slot that outgrows its place
        a(f"  .if . - {slot} > {SLOT}")
        a(f"  .error \"dispatch slot {key} is longer than {SLOT} bytes\"")
        a("  .endif")
    # ---------------------------------------------------------- end (at table + 1024 * SLOT)
    a(f"  .p2align {SLOT.bit_length() - 1}")
    a(f"{lab('end')}:")
    lane0_store("ST0", "%[outb]", SHARED)
    a("  s_waitcnt vmcnt(0)")

    body = "\n".join('        "' + line.replace('"', '\\"') + '\\n"' for line in L)
    vclob = ", ".join(f'"v{i}"' for i in range(V_CP, n_vgpr))
    sclob = ", ".join(f'"s{s[n]}"' for n in names)
    return f"""
// One 64-bit word of test cases per chunk value, held in SGPRs: S = {S} stack slots, up to {NI} inputs,
// {NP} LOAD inputs fetched ahead: s{BOOLW_SBASE}..s{BOOLW_SBASE + len(names) - 1}, v{V_CP}..v{n_vgpr - 1}.
constexpr int kBoolWordInputs = {NI};
__device__ __forceinline__ void run_boolw_dispatch_{S}(const GP_CONST uint32_t* code, const uint64_t* inb,
                                                   const uint64_t* vb, uint64_t* rb, const GP_CONST int32_t* cin,
                                                   uint32_t strideb, uint64_t* outb, uint32_t voff, uint32_t nin,
                                                   uint32_t nload, uint32_t vcoff)
{{
    const uint64_t vb64 = (uint64_t)vb, rb64 = (uint64_t)rb;
    asm volatile(
{body}
        :
        : [code] "s"(code), [inb] "s"(inb), [vb_lo] "s"((uint32_t)vb64), [vb_hi] "s"((uint32_t)(vb64 >> 32)),
          [rb_lo] "s"((uint32_t)rb64), [rb_hi] "s"((uint32_t)(rb64 >> 32)), [cin] "s"(cin),
          [strideb] "s"(strideb), [outb] "s"(outb), [voff] "v"(voff), [nin] "s"(nin), [nload] "s"(nload),
          [vcoff] "v"(vcoff)
        : "memory", "vcc", "scc", "m0", "exec", {sclob},
          {vclob});
}}
"""


def write_if_changed(path: str, text: str) -> None:
    old = open(path).read() if os.path.exists(path) else None
    if old != text:
        with open(path, "w") as fh:
            fh.write(text)


def main(out_path: str) -> None:
    head = "// Generated by gen_dispatch.py; do not edit.\n#pragma once\n"
    write_if_changed(out_path, head + "".join(gen_one(K, S, direct) for K, S in VARIANTS for direct in (False, True)))
    write_if_changed(os.path.join(os.path.dirname(out_path), "dispatch_bool.inc"),
                     head + f"constexpr int kBoolDispatchInputs = {BOOL_NI};\n"
                     + "".join(gen_bool(K, S) for K, S in BOOL_VARIANTS) + gen_bool_word())


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                                              "dispatch_f32.inc"))
