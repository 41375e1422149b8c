"""Generate the specialised SG-apply kernels (csrc/k1_gen_*.hip, csrc/k1_dispatch.inc).

For a fixed Hermite chaos (L variables, input order p_in, output order p_out)
the sparsity of the Galerkin tensor c_kij = <psi_k psi_i psi_j> and its values
are known before run time.  This script writes, per basis and precision, HIP
kernels in which the whole contraction y_i = sum_k sum_j c_kij (K_k x_j) is
unrolled: the output modes of a lane's row live in registers and every tensor
value is an immediate, so the inner loop has no table lookups.

Layout: one lane per matrix row, sliced-ELL values val[(k*7 + s)*nrows + r],
mode-major vectors.  A workgroup owns the rows of one row group (at most 64
consecutive rows).  It copies x at the distinct columns its rows reference
(the group's "halo", built on the host) into LDS with independent loads, one
tile of MT modes at a time, and contracts each tile from LDS.  Global
accesses are buffer loads/stores: a 32-bit per-lane offset (the row, or a
halo column) plus a scalar offset (the coefficient matrix and slot, or the
mode), so no 64-bit address is kept per load.

Three parameters per basis and precision keep the registers of a lane
bounded (about w (7 KC + G + 14) + 7 VGPRs, w = 1 for FP32, 2 for FP64):

* G: output modes per kernel.  P > G splits the outputs over ceil(P/G)
  kernels (output groups), each of which stages the whole halo again;
* KC: coefficient matrices per wave.  The nk matrices are split into
  ceil(nk/KC) chunks, one per wave of a workgroup; the waves' partial
  outputs are added in a fixed order through LDS (the staging buffer, reused);
* MT: modes per staging tile.  LDS holds MT x hmax values (and the partials).

Run:  python -m paper_2512_23027_amd.gen_k1   (build.py runs it)
"""

import math
import os

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
DISPATCH = os.path.join(CSRC, "k1_dispatch.inc")

# (L, p_in, p_out) -> {precision: (G, KC, MT, NW[, RG])}: the bases of the shipped
# workloads and the deterministic case (L = 0, P = 1)
BASES = {
    (0, 0, 0): {"float": (1, 1, 1, 1), "double": (1, 1, 1, 1)},
    (2, 2, 2): {"float": (6, 3, 6, 2), "double": (6, 3, 6, 2)},
    (4, 2, 3): {"float": (35, 8, 35, 2), "double": (35, 8, 35, 2)},
    (6, 2, 3): {"float": (84, 7, 32, 1), "double": (42, 7, 16, 1)},
    (8, 2, 3): {"float": (165, 6, 32, 1), "double": (83, 4, 16, 1)},
}
LDS_LIMIT = 160 * 1024

# (L, p_in, p_out) -> {precision: configuration} of the shared-halo kernels:
# every row group stages its halo in tiles of MT modes once and NW waves of
# one workgroup share it, each contracting its own coefficient matrices (at
# most KC held at a time); output groups of at most G modes are separate
# kernels (the tiled kernel of the same precision must have as many for the
# PCG variant: both write one p'q per output group); RB bytes of LDS hold
# the wave partials of one output slice.  apply: also the plain SG apply
# (else the PCG variant only).  Used when the halo fits; the tiled kernels
# of BASES otherwise.
SHARED = {
    (6, 2, 3): {"float": dict(NW=4, KC=7, MT=84, RB=40 * 1024, G=84, apply=False)},
    (8, 2, 3): {"float": dict(NW=8, KC=6, MT=165, RB=96 * 1024, G=165, apply=False)},
}


def _graded(L, p):
    out = []

    def rec(pos, rem, a):
        if pos == L - 1:
            out.append(tuple(a + [rem]))
            return
        for v in range(rem, -1, -1):
            rec(pos + 1, rem - v, a + [v])

    if L == 0:
        return [()]
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


def shape(L, p_in, p_out, T):
    """(nk, P, G, KC, MT, ngroups, nch, nw) of a basis in precision T: nch
    coefficient chunks, nw waves per workgroup (wave w takes the chunks
    c with c % nw == w, one after the other)."""
    nk, P, _ = entries(L, p_in, p_out)
    G, KC, MT, NW = BASES[(L, p_in, p_out)][T][:4]
    ngroups = (P + G - 1) // G
    G = (P + ngroups - 1) // ngroups
    nch = (nk + KC - 1) // KC
    KC = (nk + nch - 1) // nch
    nch = (nk + KC - 1) // KC
    MT = min(MT, P)
    return nk, P, G, KC, MT, ngroups, nch, min(NW, nch)


def lds_stride(MT):
    """Values per staged halo entry in LDS: MT rounded up to an odd number,
    so that the rows of a wave, whose neighbours sit at scattered entries,
    spread their reads over the LDS banks (an even stride such as 16 maps
    every entry to one of two banks and serialises the reads 32-fold)."""
    return MT if MT % 2 else MT + 1


def row_groups(L, p_in, p_out, T):
    """Row groups (64 rows each, one wave each) per workgroup: several waves
    of one workgroup run the same straight-line code in lockstep (a barrier
    per staging tile), so they share the instruction cache."""
    e = BASES[(L, p_in, p_out)][T]
    return e[4] if len(e) > 4 else 1


def tag(L, p_in, p_out):
    return "k1_L%d_%d_%d" % (L, p_in, p_out)


def kernel_source(L, p_in, p_out, T, pcg=False):
    """The output-group kernels of one basis and precision.

    pcg=True: the variant for the subdomain PCG iteration (a block whose
    active flag of iteration par is clear is skipped).  It stages
    p = z + beta p_old (beta = the block's new r'z / old r'z, 0 on the first
    iteration), writes p to pnew for its own rows (output group 0), applies
    the operator to it and writes p'q over the group's rows and the kernel's
    output modes to pqg[group * (output groups) + kernel]."""
    nk, P, ent = entries(L, p_in, p_out)
    _, _, G, KC, MT, ngroups, nch, nw = shape(L, p_in, p_out, T)
    RG = row_groups(L, p_in, p_out, T)
    S = lds_stride(MT)
    ntile = (P + MT - 1) // MT
    NT = 64 * nw * RG
    sz = "(int)sizeof(%s)" % T
    name = tag(L, p_in, p_out) + ("_pcg" if pcg else "") + ("_f" if T == "float" else "_d")
    lines = []
    for g in range(ngroups):
        i0, i1 = g * G, min(P, (g + 1) * G)
        gs = i1 - i0
        extra = (", const {T}* __restrict__ zs, {T}* __restrict__ pnew, "
                 "const double* __restrict__ rzpart, double* __restrict__ sc, int par, "
                 "double* __restrict__ pqg, unsigned long long* acct, unsigned bpr").format(T=T) if pcg else ""
        # several row groups per workgroup: two waves per SIMD (at most 256
        # registers per lane, no accumulation registers beyond them)
        lb = "%d, 2" % NT if RG > 1 else "%d" % NT
        lines.append("__global__ __launch_bounds__(%s) void %s_g%d(DEll<%s> A, DHalo H, int r0, "
                     "int nrows, const %s* __restrict__ x, int ldx, %s* __restrict__ y, int ldy, "
                     "%s alpha, %s beta, long long sx, long long sy%s) {"
                     % (lb, name, g, T, T, T, T, T, extra))
        lines.append("  extern __shared__ unsigned char k1_smem[];")
        if RG > 1:
            lines.append("  const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));")
            lines.append("  // wave wv owns row group %d blockIdx + wv and its own [hmax][%d] tile" % (RG, MT))
            lines.append("  %s* xs = reinterpret_cast<%s*>(k1_smem) + (size_t)wv * %d * H.hmax;"
                         % (T, T, S))
        elif ntile == 1:
            lines.append("  %s* xs = reinterpret_cast<%s*>(k1_smem);  // [hmax][%d] staged x" % (T, T, S))
            lines.append("  %s* part = xs + (size_t)%d * H.hmax;  // partial outputs of waves 1..%d"
                         % (T, S, nw - 1))
        else:
            lines.append("  %s* xs = reinterpret_cast<%s*>(k1_smem);  // [hmax][%d] staged tile of x;"
                         " then wave partials" % (T, T, S))
            lines.append("  %s* part = xs;" % T)
        lines.append("  const int lane = threadIdx.x & 63;")
        if RG > 1:
            lines.append("  const int graw = xcd_group(blockIdx.x, gridDim.x) * %d + wv;" % RG)
            lines.append("  const bool has = graw < H.ng;  // the last workgroup may be short")
            lines.append("  const int grp = has ? graw : 0;")
        else:
            lines.append("  const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));")
            lines.append("  const int grp = xcd_group(blockIdx.x, gridDim.x);")
        lines.append("  const int g0 = H.grow[grp], gn = H.grow[grp + 1] - g0;  // rows of this group")
        lines.append("  x += (long long)blockIdx.z * sx;")
        lines.append("  y += (long long)blockIdx.z * sy;")
        if RG > 1:
            lines.append("  const bool live = has && lane < gn && g0 + lane - r0 < nrows;")
        else:
            lines.append("  const bool live = lane < gn && g0 + lane - r0 < nrows;")
        lines.append("  const int r = g0 + (live ? lane : 0);")
        lines.append("  const int NR = A.nrows;")
        lines.append("  const auto rv = buf_rsrc(A.val), rx = buf_rsrc(x), ry = buf_rsrc(y);")
        lines.append("  const int rb = r * %s;" % sz)
        if pcg:
            lines.append("  // beta of this group's block; the block's first group stores the new r'z")
            lines.append("  const int blk = H.gblk[grp];")
            if RG > 1:
                # waves of a workgroup pass the same barriers, so a frozen
                # group's wave stays and skips its work instead of returning
                lines.append("  const bool active = __builtin_amdgcn_readfirstlane("
                             "(int)(has && sc[(size_t)blk * 8 + 2 + par] != 0.0)) != 0;")
            else:
                lines.append("  if (sc[(size_t)blk * 8 + 2 + par] == 0.0) return;  // converged block: frozen")
                lines.append("  const bool active = true;")
            lines.append("  double rzn = 0.0;")
            lines.append("  for (int j = 0; j < %d; ++j) rzn += rzpart[(size_t)blk * %d + j];" % (P, P))
            lines.append("  const double rzo = sc[(size_t)blk * 8 + 1 - par];")
            lines.append("  const %s bt = (%s)(isinf(rzo) ? 0.0 : rzn / rzo);" % (T, T))
            if g == 0:
                # one thread per row group: lane 0 of the group's wave (RG > 1)
                # or of wave 0 (the waves of a workgroup share the group)
                first = "lane == 0" if RG > 1 else "threadIdx.x == 0"
                lines.append("  if (active && %s && grp == H.bgrp[blk]) sc[(size_t)blk * 8 + par] = rzn;" % first)
                lines.append("  // algorithmic bytes of the rows this launch processes (timed launches)")
                lines.append("  if (acct && active && %s) atomicAdd(acct, (unsigned long long)gn * bpr);" % first)
            lines.append("  const auto rz = buf_rsrc(zs);")
        if RG > 1 and not pcg:
            lines.append("  const bool active = has;")
        if RG > 1:
            lines.append("  const int h0 = H.ptr[grp], nh = active ? H.ptr[grp + 1] - h0 : 0;")
        else:
            lines.append("  const int h0 = H.ptr[grp], nh = H.ptr[grp + 1] - h0;")
        lines.append("  const int rr = r - H.r0;")
        for q in range(7):
            lines.append("  const unsigned l%d = (unsigned)H.lcol[%d * H.nr + rr] * %du * %du;"
                         % (q, q, S, 4 if T == "float" else 8))
        for i in range(i0, i1):
            lines.append("  %s y%d = %s(0);" % (T, i, T))
        for t in range(ntile):
            j0, j1 = t * MT, min(P, (t + 1) * MT)
            lines.append("  // ---- tile %d: modes %d..%d" % (t, j0, j1 - 1))
            if t > 0:
                lines.append("  __syncthreads();  // every wave is done with the previous tile")
            lines.append("  for (int h = %s; h < nh; h += %d) {"
                         % ("lane" if RG > 1 else "threadIdx.x", 64 if RG > 1 else NT))
            lines.append("    const int co = H.idx[h0 + h] * %s;" % sz)
            if pcg:
                for j in range(j0, j1):
                    lines.append("    %s v%d = buf_load<%s>(rz, co, %d * ldx * %s);" % (T, j, T, j, sz))
                lines.append("    if (bt != %s(0)) {" % T)
                for j in range(j0, j1):
                    lines.append("      v%d = fma(bt, buf_load<%s>(rx, co, %d * ldx * %s), v%d);"
                                 % (j, T, j, sz, j))
                lines.append("    }")
            else:
                for j in range(j0, j1):
                    lines.append("    const %s v%d = buf_load<%s>(rx, co, %d * ldx * %s);" % (T, j, T, j, sz))
            for j in range(j0, j1):
                lines.append("    xs[h * %d + %d] = v%d;" % (S, j - j0, j))
            lines.append("  }")
            lines.append("  __syncthreads();")
            lines.append("  const char* xb%d = reinterpret_cast<const char*>(xs);" % t)
            if pcg:
                if g == 0:
                    if RG > 1:
                        lines.append("  if (active && live) {  // the new direction of the own row")
                    else:
                        lines.append("  if (wv == %d && live) {  // the new direction of the own row" % (nw - 1))
                    lines.append("    const auto rp = buf_rsrc(pnew);")
                    for j in range(j0, j1):
                        lines.append("    buf_store<%s>(*reinterpret_cast<const %s*>(xb%d + l0 + %d * sizeof(%s)), "
                                     "rp, rb, %d * ldx * %s);" % (T, T, t, j - j0, T, j, sz))
                    lines.append("  }")
            for w in range(nw):
                chunks = [ch for ch in range(nch) if ch % nw == w]
                body = []
                for ch in chunks:
                    k0, k1 = ch * KC, min(nk, (ch + 1) * KC)
                    mine = [e for e in ent if k0 <= e[0] < k1 and i0 <= e[1] < i1 and j0 <= e[2] < j1]
                    js = sorted({e[2] for e in mine})
                    if not js:
                        continue
                    ks = sorted({e[0] for e in mine})
                    body.append("    {  // coefficient matrices %d..%d" % (k0, k1 - 1))
                    if ntile > 1:
                        # an opaque zero offset per tile keeps the compiler from
                        # reusing the previous tile's loads (which would keep
                        # the matrix values live across the whole kernel)
                        body.append("    const int zk = opaque_zero();")
                    for k in ks:
                        for q in range(7):
                            body.append("    const %s k%d_%d = buf_load<%s>(rv, rb, %d * NR * %s%s);"
                                        % (T, k, q, T, k * 7 + q, sz, " + zk" if ntile > 1 else ""))
                    # straight-line modes; an empty asm statement with a memory
                    # clobber before the LDS reads of mode t+1 (issued before
                    # mode t's arithmetic, so their latency overlaps it) keeps
                    # them from being hoisted further up (live registers of two
                    # modes)
                    for q in range(7):
                        body.append("    %s n%d = *reinterpret_cast<const %s*>(xb%d + l%d + %d * sizeof(%s));"
                                    % (T, q, T, t, q, js[0] - j0, T))
                    for u, j in enumerate(js):
                        body.append("    {  // mode %d" % j)
                        for q in range(7):
                            body.append("      const %s u%d = n%d;" % (T, q, q))
                        if u + 1 < len(js):
                            body.append('      asm volatile("" ::: "memory");')
                            for q in range(7):
                                body.append("      n%d = *reinterpret_cast<const %s*>(xb%d + l%d + %d * sizeof(%s));"
                                            % (q, T, t, q, js[u + 1] - j0, T))
                        for k in sorted({e[0] for e in mine if e[2] == j}):
                            expr = "k%d_0 * u0" % k
                            for q in range(1, 7):
                                expr = "fma(k%d_%d, u%d, %s)" % (k, q, q, expr)
                            body.append("      { const %s w = %s;" % (T, expr))
                            for (_, i, _, v) in [e for e in mine if e[0] == k and e[2] == j]:
                                body.append("        y%d = fma(%s(%.17g), w, y%d);" % (i, T, v, i))
                            body.append("      }")
                        body.append("    }")
                    body.append("    }")
                if body:
                    if RG > 1:  # one chunk wave; wv numbers the row groups
                        lines.append("  if (active) {  // chunk(s) %s" % ", ".join(map(str, chunks)))
                    else:
                        lines.append("  if (wv == %d) {  // chunk(s) %s" % (w, ", ".join(map(str, chunks))))
                    lines.extend(body)
                    lines.append("  }")
        if nw > 1:
            if ntile > 1:
                lines.append("  __syncthreads();  // the staging buffer now holds the wave partials")
            lines.append("  if (wv > 0) {")
            for i in range(i0, i1):
                lines.append("    part[((wv - 1) * %d + %d) * 64 + lane] = y%d;" % (gs, i - i0, i))
            lines.append("  }")
            lines.append("  __syncthreads();")
            lines.append("  if (wv != 0) return;")
            # one wave's partials at a time (the asm statement keeps the LDS
            # reads of all waves from being issued together)
            for w in range(nw - 1):
                lines.append('  asm volatile("" ::: "memory");')
                for i in range(i0, i1):
                    lines.append("  y%d += part[(%d * %d + %d) * 64 + lane];" % (i, w, gs, i - i0))
        if RG > 1:
            lines.append("  if (!active) return;  // after the last barrier")
        lines.append("  if (live) {")
        for i in range(i0, i1):
            lines.append("    { %s v = alpha * y%d; if (beta != %s(0)) v = fma(beta, buf_load<%s>(ry, rb, %d * ldy * %s), v);"
                         " buf_store<%s>(v, ry, rb, %d * ldy * %s); }" % (T, i, T, T, i, sz, T, i, sz))
        lines.append("  }")
        if pcg:
            lines.append("  {  // p'q over this group's rows and this kernel's output modes")
            lines.append("    double v = 0.0;")
            lines.append("    if (live) {")
            for i in range(i0, i1):
                if ntile > 1 and (i - i0) % 8 == 0 and i > i0:
                    # eight modes at a time (keeps the loads from all being
                    # hoisted, which would need 2 x G registers)
                    lines.append('      asm volatile("" ::: "memory");')
                if ntile > 1:  # the own row's p, formed again as in the staging
                    lines.append("      { %s p = buf_load<%s>(rz, rb, %d * ldx * %s); if (bt != %s(0)) "
                                 "p = fma(bt, buf_load<%s>(rx, rb, %d * ldx * %s), p); "
                                 "v += (double)(alpha * y%d) * (double)p; }"
                                 % (T, T, i, sz, T, T, i, sz, i))
                else:
                    lines.append("      v += (double)(alpha * y%d) * (double)*reinterpret_cast<const %s*>(xb0 + l0 + %d * sizeof(%s));"
                                 % (i, T, i, T))
            lines.append("    }")
            lines.append("    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);")
            lines.append("    if (lane == 0) pqg[(size_t)grp * %d + %d] = v;" % (ngroups, g))
            lines.append("  }")
        lines.append("}")
        lines.append("")
    return lines, name, (nk, P, G, KC, MT, ngroups, nch, nw, NT)


def shared_cfg(L, p_in, p_out, T):
    """The shared-kernel configuration of a basis and precision, or None."""
    return SHARED.get((L, p_in, p_out), {}).get(T)


def shared_groups(L, p_in, p_out, T):
    """Output groups [(i0, i1)] of the shared kernels of a basis and precision."""
    _, P, _ = entries(L, p_in, p_out)
    G = shared_cfg(L, p_in, p_out, T)["G"]
    ng = -(-P // G)
    G = -(-P // ng)
    return [(g * G, min(P, (g + 1) * G)) for g in range(ng)]


def shared_plan(L, p_in, p_out, T, i0, i1):
    """(NW, MT, waves, R, sl) of the shared kernel of output modes [i0, i1):
    waves[w] = the sub-chunks (lists of at most KC coefficient matrices) of
    wave w, the matrices dealt to the waves by their work on these outputs
    (7 stencil products per (k, j) pair plus one product per tensor entry),
    largest first, to the least loaded wave; R output slices of sl modes for
    the reduction of the wave partials (at most RB bytes of LDS)."""
    nk, P, ent = entries(L, p_in, p_out)
    c = shared_cfg(L, p_in, p_out, T)
    NW, KC, MT, budget = c["NW"], c["KC"], c["MT"], c["RB"]
    w = 4 if T == "float" else 8
    pairs, trip = {}, {}
    for (k, i, j, v) in ent:
        if i0 <= i < i1:
            pairs.setdefault(k, set()).add(j)
            trip[k] = trip.get(k, 0) + 1
    cost = {k: 7 * len(pairs.get(k, ())) + trip.get(k, 0) for k in range(nk)}
    load = [0] * NW
    own = [[] for _ in range(NW)]
    for k in sorted(range(nk), key=lambda k: (-cost[k], k)):
        if cost[k] == 0:
            continue
        wv = min(range(NW), key=lambda q: (load[q], q))
        load[wv] += cost[k]
        own[wv].append(k)
    waves = []
    for ks in own:
        ks = sorted(ks)
        waves.append([ks[a:a + KC] for a in range(0, len(ks), KC)])
    gs = i1 - i0
    R = max(1, -(-NW * gs * 64 * w // budget))
    sl = -(-gs // R)
    R = -(-gs // sl)
    return NW, min(MT, P), waves, R, sl


UNS = 16  # staging loads in flight per thread and vector (first tile)


def shared_source(L, p_in, p_out, T, pcg, i0, i1, g):
    """The shared kernel of output modes [i0, i1) (output group g) of a
    basis and precision: the SG apply y = alpha K x + beta y over a row range,
    or (pcg) the subdomain-PCG variant that forms p = z + beta p_old while
    staging, writes p (group 0), q and the group's p'q.

    Tiles of MT modes.  Staging: the threads of the workgroup take the halo
    columns h (per threads to a column, each every per-th mode j of the
    tile), form the staged value there (x, or z + beta p_old), UNS modes at
    a time, and store it at xs[h * S + j - j0] (S odd: consecutive columns
    fall in different banks).  Products: wave w contracts its coefficient
    matrices against the tile's modes, reading the 7 neighbours of its rows
    from LDS, two modes per read.  With several tiles each wave's whole tile
    loop sits in one branch (every branch passes the same barriers).
    Reduction: for each slice of output modes every wave writes its partial
    sums to LDS (over the staged tile, no longer needed) and wave w then adds
    the partials of the slice's modes w, w + NW, ... in wave order and
    stores them; p'q of the rows is formed from the stored values and the
    own rows' p (read from LDS with one tile, else formed again from z and
    p_old as in the staging)."""
    nk, P, ent = entries(L, p_in, p_out)
    NW, MT, waves, R, sl = shared_plan(L, p_in, p_out, T, i0, i1)
    ent = [e for e in ent if i0 <= e[1] < i1]
    ntile = -(-P // MT)
    S = lds_stride(MT)
    NT = 64 * NW
    w = 4 if T == "float" else 8
    sz = "(int)sizeof(%s)" % T
    gs = i1 - i0
    M = -(-sl // NW)  # outputs per wave and slice
    # modes per run of LDS reads: two consecutive modes of a neighbour in one
    # two-address read (FP32); one in FP64, whose registers are twice as wide
    RUN = 2 if T == "float" else 1
    name = tag(L, p_in, p_out) + ("_pcg" if pcg else "") + ("_f" if T == "float" else "_d") \
        + "_s%d" % g
    out = []
    a = out.append
    if pcg:
        sig = ("DEll<%s> A, DHalo H, int nrows, const %s* __restrict__ x, int ldx, "
               "%s* __restrict__ y, int ldy, const %s* __restrict__ zs, %s* __restrict__ pnew, "
               "const double* __restrict__ rzpart, double* __restrict__ sc, int par, "
               "double* __restrict__ pqg, int ngq, unsigned long long* acct, unsigned bpr"
               % (T, T, T, T, T))
    else:
        sig = ("DEll<%s> A, DHalo H, int r0, int nrows, const %s* __restrict__ x, int ldx, "
               "%s* __restrict__ y, int ldy, %s alpha, %s beta, long long sx, long long sy"
               % (T, T, T, T, T))
    a("__global__ __launch_bounds__(%d, %d) void %s(%s) {" % (NT, max(1, 8 // NW), name, sig))
    a("  extern __shared__ unsigned char k1_smem[];")
    a("  %s* xs = reinterpret_cast<%s*>(k1_smem);  // [hmax][%d] staged tile; then the wave partials"
      % (T, T, S))
    a("  const int lane = threadIdx.x & 63;")
    a("  const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));")
    a("  const int grp = xcd_group(blockIdx.x, gridDim.x);")
    if pcg:
        a("  const int r0 = H.r0;")
        a("  const int blk = H.gblk[grp];")
        a("  if (sc[(size_t)blk * 8 + 2 + par] == 0.0) return;  // converged block: frozen (whole workgroup)")
    else:
        a("  x += (long long)blockIdx.z * sx;")
        a("  y += (long long)blockIdx.z * sy;")
    a("  const int g0 = H.grow[grp], gn = H.grow[grp + 1] - g0;  // rows of this group")
    a("  const bool live = lane < gn && g0 + lane - r0 < nrows;")
    a("  const int r = g0 + (live ? lane : 0);")
    a("  const int NR = A.nrows;")
    a("  const auto rv = buf_rsrc(A.val), rx = buf_rsrc(x), ry = buf_rsrc(y);")
    a("  const int rb = r * %s;" % sz)
    if pcg:
        a("  const auto rz = buf_rsrc(zs);")
        a("  // beta of this group's block; the block's first group stores the new r'z")
        a("  double rzn = 0.0;")
        a("  for (int j = 0; j < %d; ++j) rzn += rzpart[(size_t)blk * %d + j];" % (P, P))
        a("  const double rzo = sc[(size_t)blk * 8 + 1 - par];")
        a("  const %s bt = (%s)(isinf(rzo) ? 0.0 : rzn / rzo);" % (T, T))
        if g == 0:
            a("  if (threadIdx.x == 0 && grp == H.bgrp[blk]) sc[(size_t)blk * 8 + par] = rzn;")
            a("  // algorithmic bytes of the rows this launch processes (timed launches)")
            a("  if (acct && threadIdx.x == 0) atomicAdd(acct, (unsigned long long)gn * bpr);")
    a("  const int h0 = H.ptr[grp], nh = H.ptr[grp + 1] - h0;")
    a("  const int rr = r - H.r0;")
    for q in range(7):
        a("  const unsigned l%d = (unsigned)H.lcol[%d * H.nr + rr] * %du * %du;" % (q, q, S, w))
    a("  const char* xb = reinterpret_cast<const char*>(xs);")
    a("  // thread t stages column t % nh, modes t / nh + m * per (per threads a column)")
    a("  const int per = nh > 0 ? max(1, %d / nh) : 1, jt = nh > 0 ? (int)threadIdx.x / nh : 1;" % NT)
    for i in range(i0, i1):
        a("  %s y%d = %s(0);" % (T, i, T))

    def stage(t):
        """stage tile t in LDS (every thread of the workgroup)"""
        j0, j1 = t * MT, min(P, (t + 1) * MT)
        # later tiles stage while the accumulators are live: fewer loads in flight
        un = UNS if t == 0 else UNS // (2 if T == "float" else 4)
        a("  if (jt < per) {  // stage modes %d..%d" % (j0, j1 - 1))
        a("    for (int h = (int)threadIdx.x %% nh; h < nh; h += %d) {" % NT)
        a("      const int co = H.idx[h0 + h] * %s;" % sz)
        a("      %s* dst = xs + h * %d - %d;" % (T, S, j0))
        variants = (False, True) if pcg else (None,)
        for first in variants:
            # PCG: beta = 0 (the first iteration, p_old undefined) reads z alone
            if first is not None:
                a("      %s {" % ("if (bt != %s(0))" % T if not first else "else"))
            else:
                a("      {")
            a("        int j = %d + jt;" % j0)
            a("        for (; j + %d * per < %d; j += %d * per) {" % (un - 1, j1, un))
            a("          %s v[%d];" % (T, un))
            a("#pragma unroll")
            a("          for (int u = 0; u < %d; ++u) {" % un)
            a("            const int o = co + (j + u * per) * ldx * %s;" % sz)
            if first is None:
                a("            v[u] = buf_load<%s>(rx, o, 0);" % T)
            elif first:
                a("            v[u] = buf_load<%s>(rz, o, 0);" % T)
            else:
                a("            v[u] = fma(bt, buf_load<%s>(rx, o, 0), buf_load<%s>(rz, o, 0));" % (T, T))
            a("          }")
            a("#pragma unroll")
            a("          for (int u = 0; u < %d; ++u) dst[j + u * per] = v[u];" % un)
            a("        }")
            a("        for (; j < %d; j += per) {" % j1)
            a("          const int o = co + j * ldx * %s;" % sz)
            if first is None:
                a("          dst[j] = buf_load<%s>(rx, o, 0);" % T)
            elif first:
                a("          dst[j] = buf_load<%s>(rz, o, 0);" % T)
            else:
                a("          dst[j] = fma(bt, buf_load<%s>(rx, o, 0), buf_load<%s>(rz, o, 0));" % (T, T))
            a("        }")
            a("      }")
        a("    }")
        a("  }")

    def pnew_store(t):
        if not (pcg and g == 0):
            return
        j0, j1 = t * MT, min(P, (t + 1) * MT)
        a("  if (live) {  // the new direction of the own row: modes %d + wv, + %d, ..." % (j0, NW))
        a("    const auto rp = buf_rsrc(pnew);")
        a("    for (int j = %d + wv; j < %d; j += %d)" % (j0, j1, NW))
        a("      buf_store<%s>(*reinterpret_cast<const %s*>(xb + l0 + (j - %d) * sizeof(%s)), rp, rb, j * ldx * %s);"
          % (T, T, j0, T, sz))
        a("  }")

    def products(wq, t):
        """wave wq's contraction of its coefficient matrices with tile t"""
        j0, j1 = t * MT, min(P, (t + 1) * MT)
        for sub in waves[wq]:
            ks = set(sub)
            mine = [e for e in ent if e[0] in ks and j0 <= e[2] < j1]
            js = sorted({e[2] for e in mine})
            if not js:
                continue
            a("    {  // matrices %s, modes %d..%d" % (", ".join(map(str, sub)), j0, j1 - 1))
            if ntile > 1:
                # an opaque zero offset per tile keeps the compiler from
                # reusing the previous tile's loads (which would keep the
                # matrix values live across the whole kernel)
                a("    const int zk = opaque_zero();")
            for k in sub:
                if not any(e[0] == k for e in mine):
                    continue
                for q in range(7):
                    a("    const %s k%d_%d = buf_load<%s>(rv, rb, %d * NR * %s%s);"
                      % (T, k, q, T, k * 7 + q, sz, " + zk" if ntile > 1 else ""))
            # modes in runs of at most RUN consecutive ones
            runs = []
            for j in js:
                if runs and len(runs[-1]) < RUN and runs[-1][-1] + 1 == j:
                    runs[-1].append(j)
                else:
                    runs.append([j])

            def reads(run, decl):
                for q in range(7):
                    for b_, j in enumerate(run):
                        a("    %s%sn%d_%d = *reinterpret_cast<const %s*>(xb + l%d + %d * sizeof(%s));"
                          % ("  " if not decl else "", (T + " ") if decl else "", q, b_, T, q, j - j0, T))

            reads(runs[0], True)
            if RUN > 1 and len(runs[0]) < 2:
                for q in range(7):
                    a("    %s n%d_1 = %s(0);" % (T, q, T))
            for u, run in enumerate(runs):
                a("    {  // mode(s) %s" % ", ".join(map(str, run)))
                for b_ in range(len(run)):
                    for q in range(7):
                        a("      const %s u%d_%d = n%d_%d;" % (T, q, b_, q, b_))
                if u + 1 < len(runs):
                    # the LDS reads of the next run are issued before this
                    # run's products (the asm statement keeps them from
                    # moving further up)
                    a('      asm volatile("" ::: "memory");')
                    reads(runs[u + 1], False)
                for b_, j in enumerate(run):
                    for k in sorted({e[0] for e in mine if e[2] == j}):
                        expr = "k%d_0 * u0_%d" % (k, b_)
                        for q in range(1, 7):
                            expr = "fma(k%d_%d, u%d_%d, %s)" % (k, q, q, b_, expr)
                        a("      { const %s w = %s;" % (T, expr))
                        for (_, i, _, v) in [e for e in mine if e[0] == k and e[2] == j]:
                            a("        y%d = fma(%s(%.17g), w, y%d);" % (i, T, v, i))
                        a("      }")
                a("    }")
            # the next sub-chunk's matrix loads stay below this one's last
            # products (both sets of values live would not fit)
            a('    asm volatile("" ::: "memory");')
            a("    }")

    def head(wq):
        return "  %s (wv == %d) {  // coefficient matrices %s" % (
            "if" if wq == 0 else "} else if", wq,
            ", ".join(str(k) for sub in waves[wq] for k in sub))

    if ntile == 1:
        stage(0)
        a("  __syncthreads();")
        pnew_store(0)
        for wq in range(NW):
            a(head(wq))
            products(wq, 0)
        a("  }")
    else:
        # several tiles: each wave's whole tile loop sits in its own branch
        # (the accumulators stay in one set of registers).  Every branch
        # passes the same barriers: one after each staging, one before each
        # later staging.
        for wq in range(NW):
            a(head(wq))
            for t in range(ntile):
                if t > 0:
                    a("  __syncthreads();  // every wave is done with the previous tile")
                stage(t)
                a("  __syncthreads();")
                pnew_store(t)
                products(wq, t)
        a("  }")
    if pcg and ntile == 1:
        a("  __syncthreads();  // the products no longer read the staged p")
        a("  // own-row p of the modes this wave finalises: slice t, mode %d + t * %d + wv + %d m"
          % (i0, sl, NW))
        for t in range(R):
            s0, s1 = t * sl, min(gs, (t + 1) * sl)
            for m in range(M):
                a("  const %s po%d_%d = (wv + %d < %d) ? *reinterpret_cast<const %s*>(xb + l0 + (%d + wv + %d) * sizeof(%s)) : %s(0);"
                  % (T, t, m, NW * m, s1 - s0, T, i0 + s0, NW * m, T, T))
    if pcg:
        a("  double pq = 0.0;")
    a("  %s* part = xs;  // [wave][slice mode][64]" % T)
    for t in range(R):
        s0, s1 = t * sl, min(gs, (t + 1) * sl)
        a("  // ---- output slice %d: modes %d..%d" % (t, i0 + s0, i0 + s1 - 1))
        a("  __syncthreads();  // %s" % ("the products no longer read the staged tile" if t == 0
                                        else "the previous slice is added up"))
        for i in range(i0 + s0, i0 + s1):
            a("  part[(wv * %d + %d) * 64 + lane] = y%d;" % (sl, i - i0 - s0, i))
        a("  __syncthreads();")
        for m in range(M):
            a("  if (wv + %d < %d) {" % (NW * m, s1 - s0))
            a("    const int o = wv + %d;" % (NW * m))
            terms = ["part[(%d * %d + o) * 64 + lane]" % (q, sl) for q in range(NW)]
            a("    %s s = %s;" % (T, terms[0]))
            for tm in terms[1:]:
                a("    s += %s;" % tm)
            a("    if (live) {")
            if pcg:
                if ntile == 1:
                    a("      const %s p = po%d_%d;" % (T, t, m))
                else:
                    a("      const int so = (%d + o) * ldx * %s;" % (i0 + s0, sz))
                    a("      const %s p = bt != %s(0) ? fma(bt, buf_load<%s>(rx, rb, so), buf_load<%s>(rz, rb, so))"
                      " : buf_load<%s>(rz, rb, so);" % (T, T, T, T, T))
                a("      buf_store<%s>(s, ry, rb, (%d + o) * ldy * %s);" % (T, i0 + s0, sz))
                a("      pq += (double)s * (double)p;")
            else:
                a("      const int so = (%d + o) * ldy * %s;" % (i0 + s0, sz))
                a("      %s v = alpha * s;" % T)
                a("      if (beta != %s(0)) v = fma(beta, buf_load<%s>(ry, rb, so), v);" % (T, T))
                a("      buf_store<%s>(v, ry, rb, so);" % T)
            a("    }")
            a("  }")
    if pcg:
        a("  // p'q of the row group and this output group: wave sums, then the waves in order")
        a("  for (int o = 32; o > 0; o >>= 1) pq += __shfl_xor(pq, o, 64);")
        a("  double* pqw = reinterpret_cast<double*>(k1_smem + shared_pq_offset(H.hmax, %d, %d));"
          % (S * w, NW * sl * 64 * w))
        a("  if (lane == 0) pqw[wv] = pq;")
        a("  __syncthreads();")
        a("  if (threadIdx.x == 0) {")
        a("    double v = pqw[0];")
        for q in range(1, NW):
            a("    v += pqw[%d];" % q)
        a("    pqg[(size_t)grp * ngq + %d] = v;" % g)
        a("  }")
    a("}")
    a("")
    lds = "(shared_pq_offset(hmax, %d, %d) + %d)" % (S * w, NW * sl * 64 * w, NW * 8 if pcg else 0)
    return out, name, NT, lds


def _lds_expr(P, G, MT, ngroups, nw, T, pcg, RG=1):
    """LDS bytes of the largest output-group kernel, as a C expression of hmax."""
    gs = (P + ngroups - 1) // ngroups
    w = 4 if T == "float" else 8
    S = lds_stride(MT)
    if RG > 1:
        return "(size_t)%d * %d * hmax * %d" % (RG, S, w)
    if MT >= P:  # one tile: the partials follow the staged x
        return "((size_t)%d * hmax + %d) * %d" % (S, (nw - 1) * gs * 64, w)
    return "std::max<size_t>((size_t)%d * hmax, %d) * %d" % (S, (nw - 1) * gs * 64, w)


def basis_source(L, p_in, p_out):
    """One translation unit: the kernels of a basis in both precisions and
    their host launchers."""
    t = tag(L, p_in, p_out)
    nk, P, ent = entries(L, p_in, p_out)
    out = ["// Generated by gen_k1.py -- SG-apply kernels of the Hermite chaos L=%d, p_in=%d,"
           " p_out=%d" % (L, p_in, p_out),
           "// (%d coefficient matrices, P=%d, %d tensor entries), do not edit." % (nk, P, len(ent)),
           '#include "k1_common.h"', "", "namespace sgw {", "namespace k {", ""]
    for T in ("float", "double"):
        for pcg in (False, True):
            lines, name, (nk_, P_, G, KC, MT, ngroups, nch, nw, NT) = kernel_source(L, p_in, p_out,
                                                                                     T, pcg)
            out.append("// %s%s: %d output group(s) of <= %d modes, %d chunk(s) of <= %d coefficient"
                       " matrices on %d wave(s), tiles of %d modes"
                       % (T, " PCG" if pcg else "", ngroups, G, nch, KC, nw, MT))
            out.extend(lines)
            RG = row_groups(L, p_in, p_out, T)
            lds = _lds_expr(P, G, MT, ngroups, nw, T, pcg, RG)
            cfg = shared_cfg(L, p_in, p_out, T)
            shared = cfg is not None and (pcg or cfg["apply"])
            skern = []  # (name, threads, LDS expression) per output group
            if shared:
                sgroups = shared_groups(L, p_in, p_out, T)
                if pcg:  # both kernels write one p'q per (row group, output group)
                    assert len(sgroups) == ngroups, (L, T, len(sgroups), ngroups)
                for g, (i0, i1) in enumerate(sgroups):
                    slines, sname, SNT, slds = shared_source(L, p_in, p_out, T, pcg, i0, i1, g)
                    NW_, MT_, waves_, R_, sl_ = shared_plan(L, p_in, p_out, T, i0, i1)
                    out.append("// %s%s, shared halo, output modes %d..%d, tiles of %d modes: %d waves "
                               "(matrices %s), %d output slice(s) of %d"
                               % (T, " PCG" if pcg else "", i0, i1 - 1, MT_, NW_,
                                  " | ".join(",".join(str(k) for sub in wq for k in sub)
                                             for wq in waves_), R_, sl_))
                    out.extend(slines)
                    skern.append((sname, SNT, slds))
            smax = "std::max<size_t>({%s})" % ", ".join(k[2] for k in skern) if skern else None
            if not pcg:
                out.append("bool %s_apply(const DEll<%s>& A, const DHalo& H, int r0, int nrows, "
                           "const %s* x, int ldx, %s* y, int ldy, %s alpha, %s beta, int nbatch, "
                           "long long sx, long long sy, hipStream_t st) {" % (t, T, T, T, T, T))
                out.append("  const int ngrp = halo_groups(H, r0, nrows);")
                out.append("  const size_t hmax = H.hmax;")
                if shared:
                    out.append("  if (ngrp > 0 && %s <= %d) {  // the halo fits: shared kernels" % (smax, LDS_LIMIT))
                    for sname, SNT, slds in skern:
                        out.append("    %s<<<dim3(ngrp, 1, nbatch), %d, %s, st>>>(A, H, r0, nrows, x, ldx, "
                                   "y, ldy, alpha, beta, sx, sy);" % (sname, SNT, slds))
                    out.append("    return true;")
                    out.append("  }")
                out.append("  const size_t sh = %s;" % lds)
                out.append("  if (ngrp <= 0 || sh > %d) return false;" % LDS_LIMIT)
                out.append("  dim3 grid((ngrp + %d) / %d, 1, nbatch);" % (RG - 1, RG))
                for g in range(ngroups):
                    out.append("  %s_g%d<<<grid, %d, sh, st>>>(A, H, r0, nrows, x, ldx, y, ldy, alpha, "
                               "beta, sx, sy);" % (name, g, NT))
                out.append("  return true;")
                out.append("}")
            else:
                out.append("bool %s_pcg(const DEll<%s>& A, const DHalo& H, int nrows, const %s* pold, "
                           "const %s* zs, %s* pnew, int ld, %s* q, const double* rzpart, double* sc, "
                           "int par, double* pqg, unsigned long long* acct, unsigned bpr, "
                           "hipStream_t st) {" % (t, T, T, T, T, T))
                out.append("  const int ngrp = halo_groups(H, H.r0, nrows);")
                out.append("  const size_t hmax = H.hmax;")
                if shared:
                    out.append("  if (ngrp > 0 && %s <= %d) {  // the halo fits: shared kernels" % (smax, LDS_LIMIT))
                    for sname, SNT, slds in skern:
                        out.append("    %s<<<ngrp, %d, %s, st>>>(A, H, nrows, pold, ld, q, ld, zs, pnew, "
                                   "rzpart, sc, par, pqg, %d, acct, bpr);" % (sname, SNT, slds, ngroups))
                    out.append("    return true;")
                    out.append("  }")
                out.append("  const size_t sh = %s;" % lds)
                out.append("  if (ngrp <= 0 || sh > %d) return false;" % LDS_LIMIT)
                out.append("  dim3 grid((ngrp + %d) / %d, 1, 1);" % (RG - 1, RG))
                for g in range(ngroups):
                    out.append("  %s_g%d<<<grid, %d, sh, st>>>(A, H, H.r0, nrows, pold, ld, q, ld, "
                               "(%s)1, (%s)0, 0, 0, zs, pnew, rzpart, sc, par, pqg, acct, bpr);"
                               % (name, g, NT, T, T))
                out.append("  return true;")
                out.append("}")
            if shared:  # the kernels that run: the shared ones where they fit
                out.append("size_t %s%s_lds(%s, int hmax_i) { const size_t hmax = hmax_i; "
                           "const size_t ss = %s; return ss <= %d ? ss : %s; }"
                           % (t, "_pcg" if pcg else "", T + "*", smax, LDS_LIMIT, lds))
            else:
                out.append("size_t %s%s_lds(%s, int hmax_i) { const size_t hmax = hmax_i; return %s; }"
                           % (t, "_pcg" if pcg else "", T + "*", lds))
            out.append("")
    out.append("int %s_groups(int wbytes) { return wbytes == 4 ? %d : %d; }"
               % (t, shape(L, p_in, p_out, "float")[5], shape(L, p_in, p_out, "double")[5]))
    out.append("bool %s_prepare() {" % t)
    out.append("  bool ok = true;")
    for T in ("float", "double"):
        for pcg in (False, True):
            ngroups = shape(L, p_in, p_out, T)[5]
            name = t + ("_pcg" if pcg else "") + ("_f" if T == "float" else "_d")
            kern = ["%s_g%d" % (name, g) for g in range(ngroups)]
            cfg = shared_cfg(L, p_in, p_out, T)
            if cfg is not None and (pcg or cfg["apply"]):
                kern += ["%s_s%d" % (name, g) for g in range(len(shared_groups(L, p_in, p_out, T)))]
            for kn in kern:
                out.append("  ok = ok && hipFuncSetAttribute((const void*)%s, "
                           "hipFuncAttributeMaxDynamicSharedMemorySize, %d) == hipSuccess;"
                           % (kn, LDS_LIMIT))
    out.append("  return ok;")
    out.append("}")
    out.extend(["", "}  // namespace k", "}  // namespace sgw", ""])
    return "\n".join(out)


def dispatch_source():
    out = ["// Generated by gen_k1.py -- dispatch to the generated SG-apply kernels, do not edit.",
           "// Bases (L, p_in, p_out): " + ", ".join(str(b) for b in BASES), ""]
    for b in BASES:
        t = tag(*b)
        for T in ("float", "double"):
            out.append("bool %s_apply(const DEll<%s>&, const DHalo&, int, int, const %s*, int, %s*, "
                       "int, %s, %s, int, long long, long long, hipStream_t);" % (t, T, T, T, T, T))
            out.append("bool %s_pcg(const DEll<%s>&, const DHalo&, int, const %s*, const %s*, %s*, "
                       "int, %s*, const double*, double*, int, double*, unsigned long long*, unsigned, "
                       "hipStream_t);" % (t, T, T, T, T, T))
            out.append("size_t %s_lds(%s*, int);" % (t, T))
            out.append("size_t %s_pcg_lds(%s*, int);" % (t, T))
        out.append("int %s_groups(int);" % t)
        out.append("bool %s_prepare();" % t)
    out.append("")
    out.append("template <typename T>")
    out.append("static bool sg_apply_specialised(int L, int p_in, int p_out, const DEll<T>& A, "
               "const DHalo& H, int r0, int nrows, const T* x, int ldx, T* y, int ldy, T alpha, "
               "T beta, int nbatch, long long sx, long long sy, hipStream_t st) {")
    for b in BASES:
        out.append("  if (L == %d && p_in == %d && p_out == %d)" % b)
        out.append("    return %s_apply(A, H, r0, nrows, x, ldx, y, ldy, alpha, beta, nbatch, sx, sy, st);"
                   % tag(*b))
    out.append("  return false;")
    out.append("}")
    out.append("template <typename T>")
    out.append("static bool sg_apply_pcg_specialised(int L, int p_in, int p_out, const DEll<T>& A, "
               "const DHalo& H, int nrows, const T* pold, const T* zs, T* pnew, int ld, T* q, "
               "const double* rzpart, double* sc, int par, double* pqg, unsigned long long* acct, "
               "unsigned bpr, hipStream_t st) {")
    for b in BASES:
        out.append("  if (L == %d && p_in == %d && p_out == %d)" % b)
        out.append("    return %s_pcg(A, H, nrows, pold, zs, pnew, ld, q, rzpart, sc, par, pqg, acct, bpr, st);"
                   % tag(*b))
    out.append("  return false;")
    out.append("}")
    out.append("// LDS bytes of the generated kernel (plain or PCG variant) for a halo of")
    out.append("// hmax columns; 0 if the basis has none")
    out.append("template <typename T>")
    out.append("static size_t sg_apply_specialised_lds(int L, int p_in, int p_out, int hmax, bool pcg) {")
    for b in BASES:
        out.append("  if (L == %d && p_in == %d && p_out == %d)" % b)
        out.append("    return pcg ? %s_pcg_lds((T*)nullptr, hmax) : %s_lds((T*)nullptr, hmax);"
                   % (tag(*b), tag(*b)))
    out.append("  return 0;")
    out.append("}")
    out.append("// number of output-group kernels of the basis in a precision (4 or 8 bytes")
    out.append("// per value; 0: none generated)")
    out.append("static int sg_apply_specialised_groups(int L, int p_in, int p_out, int wbytes) {")
    for b in BASES:
        out.append("  if (L == %d && p_in == %d && p_out == %d) return %s_groups(wbytes);" % (b + (tag(*b),)))
    out.append("  return 0;")
    out.append("}")
    out.append("// Allows every generated kernel the whole 160 KiB of LDS (they have no")
    out.append("// static LDS); once per process before the first launch.")
    out.append("static bool sg_apply_specialised_prepare() {")
    out.append("  bool ok = true;")
    for b in BASES:
        out.append("  ok = ok && %s_prepare();" % tag(*b))
    out.append("  return ok;")
    out.append("}")
    return "\n".join(out) + "\n"


def sources():
    """File names of the generated translation units (relative to csrc/)."""
    return ["k1_gen_L%d_%d_%d.hip" % b for b in BASES]


def _write(path, text):
    old = open(path).read() if os.path.exists(path) else None
    if old != text:
        with open(path, "w") as f:
            f.write(text)


def generate():
    for b, f in zip(BASES, sources()):
        _write(os.path.join(CSRC, f), basis_source(*b))
    _write(DISPATCH, dispatch_source())
    return [DISPATCH] + [os.path.join(CSRC, f) for f in sources()]


if __name__ == "__main__":
    print("\n".join(generate()))
