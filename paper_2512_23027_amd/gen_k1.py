"""Generate the specialised SG-apply kernels (csrc/k1_spec.inc).

For a fixed Hermite chaos (L variables, input order p_in, output order p_out)
the sparsity of the Galerkin tensor c_kij = <psi_k psi_i psi_j> and its values
are known before run time.  This script writes one HIP kernel per such basis
in which the whole contraction y_i = sum_k sum_j c_kij (K_k x_j) is unrolled:
the output modes of a lane's row live in registers and every tensor value is
an immediate, so the inner loop has no table lookups and no LDS traffic.

Layout: one lane per matrix row, sliced-ELL values val[(k*7 + s)*nrows + r],
mode-major vectors.  A workgroup owns 64 consecutive rows; it first copies x
at the distinct columns its rows reference (the group's "halo", built on the
host, all P modes) into LDS with independent loads, then contracts from LDS.
Global accesses are buffer loads/stores: a 32-bit per-lane offset (the row,
or a halo column) plus a scalar offset (the coefficient matrix and slot, or
the mode), so no 64-bit address is kept per load.
The coefficient matrices are split into up to four chunks, one per wave of a
workgroup, so four waves share the 64 rows of a workgroup (registers per lane:
7 KC for the chunk, G for G outputs of a group, 14 for the neighbour values
of the current and the next mode, 7 halo positions); the partial outputs are
added in a fixed order through LDS.

Run:  python -m paper_2512_23027_amd.gen_k1   (build.py runs it)
"""

import math
import os

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(HERE, "csrc", "k1_spec.inc")

# (L, p_in, p_out): the bases of the shipped workloads
BASES = [(2, 2, 2), (4, 2, 3), (6, 2, 3)]
MAX_GROUP = 42         # output modes per kernel (register budget)
MAX_WAVES = 2          # waves per workgroup, one per chunk of coefficient matrices


def _graded(L, p):
    out = []

    def rec(pos, rem, a):
        if pos == L - 1:
            out.append(tuple(a + [rem]))
            return
        for v in range(rem, -1, -1):
            rec(pos + 1, rem - v, a + [v])

    for deg in range(p + 1):
        rec(0, deg, [])
    return out


def _fact(n):
    f = 1.0
    for i in range(2, n + 1):
        f *= i
    return f


def _binom(n, r):
    b = 1.0
    for i in range(1, r + 1):
        b = b * (n - r + i) / i
    return b


def _triple1(a, b, c):
    """<psi_a psi_b psi_c>, normalised 1-D Hermite, from the linearisation
    He_a He_b = sum_r C(a,r) C(b,r) r! He_{a+b-2r}."""
    twice = a + b - c
    if twice < 0 or twice % 2:
        return 0.0
    r = twice // 2
    if r > min(a, b):
        return 0.0
    e = _binom(a, r) * _binom(b, r) * _fact(r) * _fact(c)
    return e / math.sqrt(_fact(a) * _fact(b) * _fact(c))


def entries(L, p_in, p_out):
    kin, out = _graded(L, p_in), _graded(L, p_out)
    ent = []
    for k, ak in enumerate(kin):
        for i, ai in enumerate(out):
            for j, aj in enumerate(out):
                v = 1.0
                for d in range(L):
                    v *= _triple1(ak[d], ai[d], aj[d])
                    if v == 0.0:
                        break
                if v != 0.0:
                    ent.append((k, i, j, v))
    return len(kin), len(out), ent


def kernel_source(L, p_in, p_out, pcg=False):
    """One kernel per output group; a workgroup = 64 rows x NCH waves.

    pcg=True: the variant for the subdomain PCG iteration (a block whose
    active flag of iteration par is clear is skipped).  It stages
    p = z + beta p_old (beta = the block's new r'z / old r'z, 0 on the first
    iteration), writes p to pnew for its own rows, applies the operator to it
    and writes p'q over the group's rows and the kernel's output modes to
    pqg[group * (output-group kernels) + kernel].

    The workgroup first stages x at the distinct columns of its 64 rows (the
    group's halo, all P modes) in LDS with independent loads; wave w then
    contracts coefficient matrices of chunk w reading the neighbour values
    from LDS.  The partial outputs of the waves are added in a fixed order
    through LDS (the staging buffer, reused) by wave 0."""
    nk, P, ent = entries(L, p_in, p_out)
    ngroups = (P + MAX_GROUP - 1) // MAX_GROUP
    G = (P + ngroups - 1) // ngroups
    nch = min(MAX_WAVES, nk)
    KC = (nk + nch - 1) // nch
    nch = (nk + KC - 1) // KC
    NT = 64 * nch
    name = "k1_L%d_%d_%d" % (L, p_in, p_out) + ("_pcg" if pcg else "")
    lines = []
    tables = []
    for g in range(ngroups):
        i0, i1 = g * G, min(P, (g + 1) * G)
        gs = i1 - i0
        lines.append("template <typename T>")
        extra = (", const T* __restrict__ zs, T* __restrict__ pnew, const double* __restrict__ rzpart, "
                 "double* __restrict__ sc, int par, double* __restrict__ pqg") if pcg else ""
        lines.append("__global__ __launch_bounds__(%d, 2) void %s_g%d(DEll<T> A, DHalo H, int r0, int nrows, "
                     "const T* __restrict__ x, int ldx, T* __restrict__ y, int ldy, T alpha, "
                     "T beta, long long sx, long long sy%s) {" % (NT, name, g, extra))
        lines.append("  extern __shared__ unsigned char k1_smem[];")
        lines.append("  T* xs = reinterpret_cast<T*>(k1_smem);  // [halo][P] staged x")
        lines.append("  T* part = xs + (size_t)%d * H.hmax;  // partial outputs of waves 1..%d" % (P, nch - 1))
        lines.append("  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;")
        lines.append("  const int grp = xcd_group(blockIdx.x, gridDim.x);")
        lines.append("  const int g0 = H.grow[grp], gn = H.grow[grp + 1] - g0;  // rows of this group")
        lines.append("  x += (long long)blockIdx.z * sx;")
        lines.append("  y += (long long)blockIdx.z * sy;")
        lines.append("  const bool live = lane < gn && g0 + lane - r0 < nrows;")
        lines.append("  const int r = g0 + (live ? lane : 0);")
        lines.append("  const int NR = A.nrows;")
        lines.append("  const auto rv = buf_rsrc(A.val), rx = buf_rsrc(x), ry = buf_rsrc(y);")
        lines.append("  const int rb = r * (int)sizeof(T);")
        # staging: every thread owns halo entries h, loads all P modes at once
        if pcg:
            lines.append("  // beta of this group's block; the block's first group stores the new r'z")
            lines.append("  const int blk = H.gblk[grp];")
            lines.append("  if (sc[(size_t)blk * 8 + 2 + par] == 0.0) return;  // converged block: frozen")
            lines.append("  double rzn = 0.0;")
            lines.append("  for (int j = 0; j < %d; ++j) rzn += rzpart[(size_t)blk * %d + j];" % (P, P))
            lines.append("  const double rzo = sc[(size_t)blk * 8 + 1 - par];")
            lines.append("  const T bt = (T)(isinf(rzo) ? 0.0 : rzn / rzo);")
            lines.append("  if (threadIdx.x == 0 && grp == H.bgrp[blk]) sc[(size_t)blk * 8 + par] = rzn;")
            lines.append("  const auto rz = buf_rsrc(zs);")
        lines.append("  {")
        lines.append("    const int h0 = H.ptr[grp], nh = H.ptr[grp + 1] - h0;")
        lines.append("    for (int h = threadIdx.x; h < nh; h += %d) {" % NT)
        lines.append("      const int co = H.idx[h0 + h] * (int)sizeof(T);")
        if pcg:
            for j in range(P):
                lines.append("      T v%d = buf_load<T>(rz, co, %d * ldx * (int)sizeof(T));" % (j, j))
            lines.append("      if (bt != T(0)) {")
            for j in range(P):
                lines.append("        v%d = fma(bt, buf_load<T>(rx, co, %d * ldx * (int)sizeof(T)), v%d);" % (j, j, j))
            lines.append("      }")
        else:
            for j in range(P):
                lines.append("      const T v%d = buf_load<T>(rx, co, %d * ldx * (int)sizeof(T));" % (j, j))
        for j in range(P):
            lines.append("      xs[h * %d + %d] = v%d;" % (P, j, j))
        lines.append("    }")
        lines.append("  }")
        lines.append("  const int rr = r - H.r0;")
        for q in range(7):
            lines.append("  const unsigned l%d = (unsigned)H.lcol[%d * H.nr + rr] * %du * (unsigned)sizeof(T);" % (q, q, P))
        for i in range(i0, i1):
            lines.append("  T y%d = T(0);" % i)
        lines.append("  __syncthreads();")
        if pcg and g == 0:
            lines.append("  if (wv == %d && live) {  // the new direction of the own row" % (nch - 1))
            lines.append("    const auto rp = buf_rsrc(pnew);")
            lines.append("    const char* xb0 = reinterpret_cast<const char*>(xs);")
            for j in range(P):
                lines.append("    buf_store<T>(*reinterpret_cast<const T*>(xb0 + l0 + %d * sizeof(T)), rp, rb, %d * ldx * (int)sizeof(T));" % (j, j))
            lines.append("  }")
        for ch in range(nch):
            k0, k1 = ch * KC, min(nk, (ch + 1) * KC)
            mine = [e for e in ent if k0 <= e[0] < k1 and i0 <= e[1] < i1]
            js = [j for j in range(P) if any(e[2] == j for e in mine)]
            if not js:
                continue
            lines.append("  if (wv == %d) {  // coefficient matrices %d..%d" % (ch, k0, k1 - 1))
            for k in range(k0, k1):
                for q in range(7):
                    lines.append("    const T k%d_%d = buf_load<T>(rv, rb, %d * NR * (int)sizeof(T));"
                                 % (k, q, k * 7 + q))
            # The modes of this chunk run as straight-line code.  An empty asm
            # statement with a memory clobber before the LDS reads of mode
            # t+1 (issued before mode t's arithmetic, so their latency
            # overlaps it) keeps them from being hoisted further up, which
            # keeps the live registers those of two modes.
            lines.append("    const char* xb = reinterpret_cast<const char*>(xs);")
            for q in range(7):
                lines.append("    T n%d = *reinterpret_cast<const T*>(xb + l%d + %d * sizeof(T));" % (q, q, js[0]))
            for t, j in enumerate(js):
                lines.append("    {  // mode %d" % j)
                for q in range(7):
                    lines.append("      const T u%d = n%d;" % (q, q))
                if t + 1 < len(js):
                    lines.append('      asm volatile("" ::: "memory");')
                    for q in range(7):
                        lines.append("      n%d = *reinterpret_cast<const T*>(xb + l%d + %d * sizeof(T));"
                                     % (q, q, js[t + 1]))
                for k in sorted({e[0] for e in mine if e[2] == j}):
                    expr = "k%d_0 * u0" % k
                    for q in range(1, 7):
                        expr = "fma(k%d_%d, u%d, %s)" % (k, q, q, expr)
                    lines.append("      { const T w = %s;" % expr)
                    for (_, i, _, v) in [e for e in mine if e[0] == k and e[2] == j]:
                        lines.append("        y%d = fma(T(%.17g), w, y%d);" % (i, v, i))
                    lines.append("      }")
                lines.append("    }")
            lines.append("  }")
        if nch > 1:
            lines.append("  if (wv > 0) {")
            for i in range(i0, i1):
                lines.append("    part[((wv - 1) * %d + %d) * 64 + lane] = y%d;" % (gs, i - i0, i))
            lines.append("  }")
            lines.append("  __syncthreads();")
            lines.append("  if (wv != 0) return;")
            for i in range(i0, i1):
                lines.append("  y%d = %s;" % (i, " + ".join(["y%d" % i] + ["part[(%d * %d + %d) * 64 + lane]"
                                                                       % (w, gs, i - i0)
                                                                       for w in range(nch - 1)])))
        lines.append("  if (live) {")
        for i in range(i0, i1):
            lines.append("    { T v = alpha * y%d; if (beta != T(0)) v = fma(beta, buf_load<T>(ry, rb, %d * ldy * (int)sizeof(T)), v);"
                         " buf_store<T>(v, ry, rb, %d * ldy * (int)sizeof(T)); }" % (i, i, i))
        lines.append("  }")
        if pcg:
            lines.append("  {  // p'q over this group's rows and this kernel's output modes")
            lines.append("    const char* xb0 = reinterpret_cast<const char*>(xs);")
            lines.append("    double v = 0.0;")
            lines.append("    if (live) {")
            for i in range(i0, i1):
                lines.append("      v += (double)(alpha * y%d) * (double)*reinterpret_cast<const T*>(xb0 + l0 + %d * sizeof(T));" % (i, i))
            lines.append("    }")
            lines.append("    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);")
            lines.append("    if (lane == 0) pqg[(size_t)grp * %d + %d] = v;" % (ngroups, g))
            lines.append("  }")
        lines.append("}")
        lines.append("")
    # dispatcher: one workgroup per row group of the halo that starts at r0
    xsig = (", const T* zs, T* pnew, const double* rzpart, double* sc, int par, double* pqg"
            if pcg else "")
    xarg = ", zs, pnew, rzpart, sc, par, pqg" if pcg else ""
    lines.append("template <typename T>")
    lines.append("static void %s_launch(const DEll<T>& A, const DHalo& H, int r0, int nrows, const T* x, "
                 "int ldx, T* y, int ldy, T alpha, T beta, int nbatch, long long sx, long long sy%s, "
                 "hipStream_t st) {" % (name, xsig))
    lines.append("  const int ngrp = halo_groups(H, r0, nrows);")
    lines.append("  if (ngrp <= 0) return;")
    lines.append("  dim3 grid(ngrp, 1, nbatch);")
    for g in range(ngroups):
        gs = min(P, (g + 1) * G) - g * G
        lines.append("  {")
        lines.append("    const size_t sh = sizeof(T) * ((size_t)%d * H.hmax + %d);" % (P, (nch - 1) * gs * 64))
        lines.append("    %s_g%d<T><<<grid, %d, sh, st>>>(A, H, r0, nrows, x, ldx, y, ldy, alpha, beta, sx, sy%s);"
                     % (name, g, NT, xarg))
        lines.append("  }")
    lines.append("}")
    lines.append("")
    # LDS attribute for every kernel of this basis
    lines.append("static bool %s_prepare() {" % name)
    lines.append("  bool ok = true;")
    for g in range(ngroups):
        for T in ("float", "double"):
            lines.append("  ok = ok && hipFuncSetAttribute((const void*)%s_g%d<%s>, "
                         "hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024) == hipSuccess;"
                         % (name, g, T))
    lines.append("  return ok;")
    lines.append("}")
    lines.append("")
    return "\n".join(tables + [""] + lines), name, nk, P, len(ent)


def max_lds_modes():
    """Largest P among the generated bases (the staged x holds P x hmax)."""
    return max(entries(*b)[1] for b in BASES)


def generate():
    parts = ["// Generated by gen_k1.py -- specialised SG-apply kernels, do not edit.",
             "// Bases (L, p_in, p_out): " + ", ".join(str(b) for b in BASES), ""]
    disp = ["template <typename T>",
            "static bool sg_apply_specialised(int L, int p_in, int p_out, const DEll<T>& A, "
            "const DHalo& H, int r0, int nrows, const T* x, int ldx, T* y, int ldy, T alpha, "
            "T beta, int nbatch, long long sx, long long sy, hipStream_t st) {"]
    prep = ["// Allows every generated kernel the whole 160 KiB of LDS (they have no",
            "// static LDS); once per process before the first launch.",
            "static bool sg_apply_specialised_prepare() {",
            "  bool ok = true;"]
    dpcg = ["template <typename T>",
            "static bool sg_apply_pcg_specialised(int L, int p_in, int p_out, const DEll<T>& A, "
            "const DHalo& H, int nrows, const T* pold, const T* zs, T* pnew, int ld, T* q, "
            "const double* rzpart, double* sc, int par, double* pqg, hipStream_t st) {"]
    for (L, pi, po) in BASES:
        src, name, nk, P, nnz = kernel_source(L, pi, po)
        srcp, namep, _, _, _ = kernel_source(L, pi, po, pcg=True)
        parts.append("// L=%d p_in=%d p_out=%d: %d coefficient matrices, P=%d, %d tensor entries"
                     % (L, pi, po, nk, P, nnz))
        parts.append(src)
        parts.append(srcp)
        disp.append("  if (L == %d && p_in == %d && p_out == %d) {" % (L, pi, po))
        disp.append("    %s_launch<T>(A, H, r0, nrows, x, ldx, y, ldy, alpha, beta, nbatch, sx, sy, st);"
                    % name)
        disp.append("    return true;")
        disp.append("  }")
        dpcg.append("  if (L == %d && p_in == %d && p_out == %d) {" % (L, pi, po))
        dpcg.append("    %s_launch<T>(A, H, H.r0, nrows, pold, ld, q, ld, T(1), T(0), 1, 0, 0, zs, pnew, "
                    "rzpart, sc, par, pqg, st);" % namep)
        dpcg.append("    return true;")
        dpcg.append("  }")
        prep.append("  ok = ok && %s_prepare();" % name)
        prep.append("  ok = ok && %s_prepare();" % namep)
    disp.append("  return false;")
    disp.append("}")
    dpcg.append("  return false;")
    dpcg.append("}")
    disp.append("")
    disp.extend(dpcg)
    disp.append("")
    disp.append("// number of output-group kernels of the basis (0: none generated)")
    disp.append("static int sg_apply_specialised_groups(int L, int p_in, int p_out) {")
    for (L, pi, po) in BASES:
        P = entries(L, pi, po)[1]
        ng = (P + MAX_GROUP - 1) // MAX_GROUP
        disp.append("  if (L == %d && p_in == %d && p_out == %d) return %d;" % (L, pi, po, ng))
    disp.append("  return 0;")
    disp.append("}")
    prep.append("  return ok;")
    prep.append("}")
    parts.extend(disp)
    parts.append("")
    parts.extend(prep)
    text = "\n".join(parts) + "\n"
    old = open(OUT).read() if os.path.exists(OUT) else None
    if old != text:
        with open(OUT, "w") as f:
            f.write(text)
    return OUT


if __name__ == "__main__":
    print(generate())
