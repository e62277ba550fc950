"""Generates the HIP right-hand side of a mass-action network.

The generated code fixes the network's topology (species count and which
species fill each reactant / product slot) at compile time, so every species
index is a constant and the per-system state stays in registers.  Rate
parameters (ln A, b, E, 1/K) and molar masses stay runtime data: they are read
from a uniform device buffer laid out as

    [lnA (n_rx) | beta (n_rx) | Ea (n_rx) | invK (n_rx) | W (n_sp) | invW (n_sp)]

Rate law (Sec. 4.2 species equations with this project's network convention):
C_k = (rho Y_k) / W_k, [M] = sum_k C_k,
q_j = k_f,j prod_R C - k_r,j prod_P C, a one-species side times [M],
k_r,j = k_f,j (1 / K_j), dY_k/dt = (W_k sum_j nu_kj q_j) / rho, with
k_f,j = exp(lnA_j + b_j ln T - E_j / T) formed once per system; divisions by
constants are multiplications by reciprocals formed once.
"""
from __future__ import annotations

import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
GEN_DIR = os.path.join(HERE, "csrc", "gen")


def _side(coef, slots):
    a, b = int(slots[0]), int(slots[1])
    second = f"C[{b}]" if b >= 0 else "M"
    return f"({coef} * C[{a}]) * {second}"


# Networks with at most this many species keep their vectors in registers
# (rate constants too); larger ones keep every vector and the rate constants
# in slot columns of the device workspace.
REGISTER_SPECIES_LIMIT = 16
# Larger networks also get a group variant in which several lanes share a
# system: 16 lanes up to 32 species, 32 lanes above.


def group_lanes(n_sp: int) -> int:
    return 16 if n_sp <= 32 else 32


def _gershgorin_source(net) -> str:
    """Gershgorin bound max_k sum_i |J_ki| of the analytic Jacobian at y, in
    the reference evaluation's order: C and [M] as in the right-hand side;
    J_ki = (W_k D_ki) (1/W_i), D_ki the sum over the reactions in order with
    nu_kj != 0 of nu_kj g_ji, g_ji = k_f t_f - k_r t_r, t_f = [r0 = i] X_r1 +
    [r1 = i or empty] C_r0 (t_r likewise); rows summed over i from zero, the
    maximum by fmax from zero.  Entries and terms that are zero by structure
    are left out (adding a zero changes no sum here)."""
    n, nr = net.n_sp, net.n_rx
    lines = ["  static constexpr bool kGershgorin = true;",
             "  template <class VI>",
             "  RKMI_HD static double gershgorin(const Lane& L, const Params& p, const VI& y) {",
             "    const double* __restrict__ iK = p + 3 * NR;",
             "    const double* __restrict__ W = p + 4 * NR;",
             "    const double* __restrict__ iW = W + N;",
             "    const int z = opaque_zero();",
             "    double C[N];",
             "#pragma unroll",
             "    for (int k = 0; k < N; ++k) C[k] = (L.rho * y[k]) * ld_uniform(iW, k);",
             "    double M = 0.0;",
             "#pragma unroll",
             "    for (int k = 0; k < N; ++k) M += C[k];",
             "    double sigma = 0.0;"]

    def x(s):
        return f"C[{s}]" if s >= 0 else "M"
    for k in range(n):
        rx = []
        for j in range(nr):
            r0, r1 = int(net.reac[j][0]), int(net.reac[j][1])
            p0, p1 = int(net.prod[j][0]), int(net.prod[j][1])
            nu = (p0 == k) + (p1 == k) - (r0 == k) - (r1 == k)
            if nu:
                rx.append((j, nu, r0, r1, p0, p1))
        lines.append("    {")
        for j, *_ in rx:
            lines.append(f"      const double kf{j} = L.kf[z + {j} * kLdsStride];")
            lines.append(f"      const double kr{j} = kf{j} * ld_uniform(iK, {j});")
        lines.append("      double r = 0.0;")
        for i in range(n):
            terms = []
            for j, nu, r0, r1, p0, p1 in rx:
                tf = ([x(r1)] if r0 == i else []) + ([x(r0)] if (r1 < 0 or r1 == i) else [])
                tr = ([x(p1)] if p0 == i else []) + ([x(p0)] if (p1 < 0 or p1 == i) else [])
                if not tf and not tr:
                    continue
                fs = f"kf{j} * ({' + '.join(tf)})" if tf else None
                rs = f"kr{j} * ({' + '.join(tr)})" if tr else None
                g = f"{fs} - {rs}" if fs and rs else (fs if fs else f"-({rs})")
                terms.append({1: f"({g})", -1: f"-({g})", 2: f"2.0 * ({g})",
                              -2: f"-2.0 * ({g})"}[nu])
            if terms:
                lines.append(f"      r += fabs((ld_uniform(W, {k}) * ({' + '.join(terms)})) * "
                             f"ld_uniform(iW, {i}));")
        lines.append("      sigma = fmax(sigma, r);")
        lines.append("    }")
    lines += ["    return sigma;", "  }"]
    return "\n".join(lines) + "\n"


def rhs_source(net, tag: str) -> tuple[str, str]:
    """Every operation is written in the order of the reference evaluation
    (products left to right, rate of progress as forward minus reverse, species
    sums accumulated reaction by reaction from zero), and the library is built
    without floating-point contraction, so each rounding is the same."""
    n, nr = net.n_sp, net.n_rx
    columns = n > REGISTER_SPECIES_LIMIT
    lines = []
    for j in range(nr):
        r, p = net.reac[j], net.prod[j]
        lines.append(f"    kf = L.kf[{j} * kLdsStride];" if columns else f"    kf = L.kf[z + {j} * kLdsStride];")
        lines.append(f"    kr = kf * ld_uniform(iK, {j});")
        lines.append(f"    q = {_side('kf', r)} - {_side('kr', p)};")
        for k in r:
            if k >= 0:
                lines.append(f"    om[{int(k)}] -= q;")
        for k in p:
            if k >= 0:
                lines.append(f"    om[{int(k)}] += q;")
    body = "\n".join(lines)
    vjp = "" if columns else _vjp_source(net) + _gershgorin_source(net)
    group = group_source(net, tag) if columns else ""
    fast = (f"template <>\nstruct FastVariant<gen_{tag}::Net> {{\n  using type = gen_{tag}::GNet;\n}};\n\n"
            if columns else "")
    if columns:
        launch_call = (f"rkmi::launch_with_group<rkmi::gen_{tag}::Net, rkmi::gen_{tag}::GNet>(a, s)")
        ws_call = (f"rkmi::workspace_with_group<rkmi::gen_{tag}::Net, rkmi::gen_{tag}::GNet>"
                   "(method, schedule, n)")
    else:
        launch_call = f"rkmi::launch<rkmi::gen_{tag}::Net>(a, s)"
        ws_call = f"rkmi::workspace<rkmi::gen_{tag}::Net>(method, schedule, n)"
    if columns:
        storage = """  // vectors and the forward rate constants k_f,j of the system live in slot
  // columns (stride kLdsStride); each k_f,j is read once per evaluation
  static constexpr bool kColumns = true;
  static constexpr int kGroupLanes = 1;
  static constexpr int kLaneDoubles = NR;
  using Params = const double*;
  struct Lane {
    const double* kf;
    double rho, irho;
  };"""
        fill = """    for (int j = 0; j < NR; ++j)
      slot[j * kLdsStride] = crm::cr_exp(p[j] + p[NR + j] * lnT - p[2 * NR + j] / T);
    L.kf = slot;"""
    else:
        storage = """  // vectors live in registers; the forward rate constants k_f,j of the
  // system live in the lane's LDS slot and are read once per evaluation (at an
  // offset the optimizer cannot see through, so the reads and the reverse
  // constants k_f,j / K_j are not hoisted out of the integration loop into
  // ~100 live registers)
  static constexpr bool kColumns = false;
  static constexpr int kGroupLanes = 1;
  static constexpr int kLaneDoubles = NR;
  // two waves per SIMD (the slot, NR + N doubles per lane, fits eight
  // workgroups in a compute unit's LDS up to 13 species and 27 reactions)
  static constexpr int kWavesPerEu = 2;
  using Params = const double*;
  struct Lane {
    const double* kf;
    double rho, irho;
  };"""
        fill = """#pragma nounroll
    for (int j = 0; j < NR; ++j)
      slot[j * kLdsStride] = crm::cr_exp(p[j] + p[NR + j] * lnT - p[2 * NR + j] / T);
    L.kf = slot;"""
    zdecl = "" if columns else "    const int z = opaque_zero();\n"
    header = f"""// Generated by paper_1611_02274_amd/codegen.py -- do not edit.
// Mass-action network: {n} species, {nr} reversible reactions (topology {tag}).
#pragma once

#include "../rk_adjoint.hpp"
#include "../rk_group.hpp"

namespace rkmi {{
namespace gen_{tag} {{

struct Net {{
  static constexpr int N = {n};
  static constexpr int NR = {nr};
{storage}
  RKMI_HD static void init(Lane& L, const Params& p, const double* __restrict__ g, int64_t i,
                           int64_t n, double* slot) {{
    const double T = g[i];
    const double rho = g[n + i];
    const double lnT = crm::cr_log(T);
{fill}
    L.rho = rho;
    L.irho = 1.0 / rho;
  }}
  template <class VI, class VO>
  RKMI_HD static void rhs(const Lane& L, const Params& p, const VI& y, VO& f) {{
    const double* __restrict__ iK = p + 3 * NR;
    const double* __restrict__ W = p + 4 * NR;
    const double* __restrict__ iW = W + N;
    double C[N], om[N];
{zdecl}#pragma unroll
    for (int k = 0; k < N; ++k) C[k] = (L.rho * y[k]) * ld_uniform(iW, k);
    double M = 0.0;
#pragma unroll
    for (int k = 0; k < N; ++k) M += C[k];
#pragma unroll
    for (int k = 0; k < N; ++k) om[k] = 0.0;
    double q, kf, kr;
{body}
#pragma unroll
    for (int k = 0; k < N; ++k) f[k] = (ld_uniform(W, k) * om[k]) * L.irho;
  }}
{vjp}}};
{group}
}}  // namespace gen_{tag}

{fast}}}  // namespace rkmi
"""
    source = f"""// Generated by paper_1611_02274_amd/codegen.py -- do not edit.
// Launchers of the {n}-species network (topology {tag}).
#include "net_{tag}.hpp"

extern "C" int rkmi_gen_{tag}_launch(const rkmi::LaunchArgs* a, void* s) {{
  return {launch_call};
}}

extern "C" int rkmi_gen_{tag}_host(const rkmi::LaunchArgs* a) {{
  return rkmi::host_run<rkmi::gen_{tag}::Net>(a);
}}

extern "C" int64_t rkmi_gen_{tag}_workspace(int method, int schedule, int64_t n) {{
  return {ws_call};
}}
{"" if columns else _adjoint_exports(tag)}"""
    return header, source


def thermal_source(net, tag: str) -> tuple[str, str]:
    """The network with the energy equation (Sec. 4.2 at constant volume):
    state (T, Y_1..Y_N), one parameter per system (rho); the rate coefficients
    are evaluated at the current T in every evaluation (a rolled loop through
    the lane's LDS slot, one copy of the exponential's code), the species part
    is the isothermal rate law, and dT/dt = -((sum_k (e_k omega_k) W_k / rho) /
    c_v).  Same operations in the same order as the reference evaluation.
    Systems of up to 16 unknowns keep their vectors in registers."""
    n, nr = net.n_sp, net.n_rx
    assert n + 1 <= REGISTER_SPECIES_LIMIT
    lines = []
    for j in range(nr):
        r, p = net.reac[j], net.prod[j]
        lines.append(f"    kf = L.kf[z + {j} * kLdsStride];")
        lines.append(f"    kr = kf * ld_uniform(iK, {j});")
        lines.append(f"    q = {_side('kf', r)} - {_side('kr', p)};")
        for k in r:
            if k >= 0:
                lines.append(f"    om[{int(k)}] -= q;")
        for k in p:
            if k >= 0:
                lines.append(f"    om[{int(k)}] += q;")
    body = "\n".join(lines)
    header = f"""// Generated by paper_1611_02274_amd/codegen.py -- do not edit.
// Mass-action network with the energy equation: {n} species + T, {nr} reversible
// reactions (topology {tag}).
#pragma once

#include "../rk_launch.hpp"

namespace rkmi {{
namespace gen_{tag} {{

struct Net {{
  static constexpr int NS = {n};
  static constexpr int N = NS + 1;
  static constexpr int NR = {nr};
  // vectors in registers; k_f,j(T) of the current evaluation in the lane's LDS
  // slot, read back at an offset the optimizer cannot see through
  static constexpr bool kColumns = false;
  static constexpr int kGroupLanes = 1;
  static constexpr int kLaneDoubles = NR;
  static constexpr int kWavesPerEu = 2;
  // uniform data: [lnA | beta | Ea | 1/K | W | 1/W | u0 | cv0 | cv1]
  using Params = const double*;
  struct Lane {{
    double* kf;
    double rho, irho;
  }};
  RKMI_HD static void init(Lane& L, const Params&, const double* __restrict__ g, int64_t i,
                           int64_t, double* slot) {{
    L.kf = slot;
    L.rho = g[i];
    L.irho = 1.0 / L.rho;
  }}
  template <class VI, class VO>
  RKMI_HD static void rhs(const Lane& L, const Params& p, const VI& y, VO& f) {{
    const double* __restrict__ iK = p + 3 * NR;
    const double* __restrict__ W = p + 4 * NR;
    const double* __restrict__ iW = W + NS;
    const double* __restrict__ u0 = W + 2 * NS;
    const double* __restrict__ cv0 = W + 3 * NS;
    const double* __restrict__ cv1 = W + 4 * NS;
    const double T = y[0];
    const double lnT = crm::cr_log(T);
    const double invT = 1.0 / T;
    const int z = opaque_zero();
    // three exps in flight per iteration (their table gathers overlap; measured
    // 6 % over a rolled loop, two waves per SIMD)
#pragma unroll 3
    for (int j = 0; j < NR; ++j)
      L.kf[z + j * kLdsStride] = crm::cr_exp(ld_uniform(p, j) + ld_uniform(p, NR + j) * lnT -
                                             ld_uniform(p, 2 * NR + j) * invT);
    double C[NS], om[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) C[k] = (L.rho * y[1 + k]) * ld_uniform(iW, k);
    double M = 0.0;
#pragma unroll
    for (int k = 0; k < NS; ++k) M += C[k];
#pragma unroll
    for (int k = 0; k < NS; ++k) om[k] = 0.0;
    double q, kf, kr;
{body}
#pragma unroll
    for (int k = 0; k < NS; ++k) f[1 + k] = (ld_uniform(W, k) * om[k]) * L.irho;
    double sum = 0.0, cv = 0.0;
#pragma unroll
    for (int k = 0; k < NS; ++k) {{
      const double e = ld_uniform(u0, k) + (ld_uniform(cv0, k) + ld_uniform(cv1, k) * T) * T;
      sum += (e * om[k]) * ld_uniform(W, k);
      cv += y[1 + k] * (ld_uniform(cv0, k) + 2.0 * ld_uniform(cv1, k) * T);
    }}
    f[0] = -((sum * L.irho) / cv);
  }}
}};

}}  // namespace gen_{tag}
}}  // namespace rkmi
"""
    source = f"""// Generated by paper_1611_02274_amd/codegen.py -- do not edit.
// Launchers of the {n}-species network with the energy equation (topology {tag}).
#include "net_{tag}.hpp"

extern "C" int rkmi_gen_{tag}_launch(const rkmi::LaunchArgs* a, void* s) {{
  return rkmi::launch<rkmi::gen_{tag}::Net>(a, s);
}}

extern "C" int rkmi_gen_{tag}_host(const rkmi::LaunchArgs* a) {{
  return rkmi::host_run<rkmi::gen_{tag}::Net>(a);
}}

extern "C" int64_t rkmi_gen_{tag}_workspace(int method, int schedule, int64_t n) {{
  return rkmi::workspace<rkmi::gen_{tag}::Net>(method, schedule, n);
}}
"""
    return header, source


def thermal_group_source(net, tag: str) -> tuple[str, str]:
    """The network with the energy equation on the group schedule (32 lanes
    per system, rk_group.hpp group_rhs_thermal): unknowns (T, Y_1..Y_N) over the
    lanes' slots, the rate coefficients k_f,j(T) formed by each position's lane
    at every evaluation, the species part as the isothermal group right-hand
    side, and dT/dt from two species sums passed along the chain of lanes.
    Same operations in the same order as the reference evaluation."""
    n, nr = net.n_sp, net.n_rx
    G = _group_layout(net, 32, thermal=True)
    header = f"""// Generated by paper_1611_02274_amd/codegen.py -- do not edit.
// Mass-action network with the energy equation on the group schedule: {n} species
// + T, {nr} reversible reactions (topology {tag}).
#pragma once

#include "../rk_launch.hpp"
#include "../rk_group.hpp"

namespace rkmi {{
namespace gen_{tag} {{

struct GNet {{
  static constexpr bool kThermal = true;
  static constexpr int NS = {n};
  static constexpr int N = NS + 1;    // unknowns: T, then the species
  static constexpr int NR = {nr};
  static constexpr int kL = {G["L"]};
  static constexpr int kGroupLanes = {G["L"]};
  static constexpr bool kColumns = false;
  static constexpr int kLaneDoubles = 0;
  static constexpr int kWavesPerEuRkc = 2;
  static constexpr int kWavesPerEuRkck = 2;
  static constexpr int S = {G["S"]};
  static constexpr int R = {G["R"]};
  static constexpr int kMSlot = {G["m_first"]};   // first slot that may hold a [M] reaction
  static constexpr int kOffC = 0;
  static constexpr int kOffT = NS + 1;            // T, written by its owner
  static constexpr int kOffQ = {G["off_q"]};
  static constexpr int kSentinel = {G["sentinel"]};
  static constexpr int kNegOff = {G["neg"]};
  static constexpr int kOffRed = {G["off_red"]};
  static constexpr int kOffE1 = {G["off_e1"]};   // the energy sum's terms (after the RKC coefficients)
  static constexpr int kOffE2 = {G["off_e2"]};   // the heat capacity's terms
  static constexpr int kLdsPerSystem = {G["lds_per_system"]};
  static constexpr int kTermBits = {G["bits"]};
  static constexpr int kTermsPerWord = {G["per_word"]};
  static constexpr int kTermWords = {G["n_words"]};
  static constexpr int kTermLen = {G["tot"]};
  static constexpr int kChunk = {G["chunk"]};
  // uniform data: [lnA | beta | Ea | 1/K | W | 1/W | u0 | cv0 | cv1]
  using Params = const double*;
{_group_tables(G)}
  struct Lane {{
    const double* prm;   // the uniform data (rate parameters read at every evaluation)
    double W[S], iW[S], u0[S], cv0[S], cv1[S];
    double rho, irho;
    int bnd;   // chunks of the slot-0 list
  }};
  __device__ static void init(Lane& L, const Params& p, const double* __restrict__ g, int64_t i,
                              int64_t, const Grp<GNet>& x) {{
    L.prm = p;
#pragma unroll
    for (int m = 0; m < S; ++m) {{
      const int k = x.sp[m] - 1;   // species of the slot (T and empty slots: none)
      const bool sp = k >= 0;
      L.W[m] = sp ? p[4 * NR + k] : 0.0;
      L.iW[m] = sp ? p[4 * NR + NS + k] : 0.0;
      L.u0[m] = sp ? p[4 * NR + 2 * NS + k] : 0.0;
      L.cv0[m] = sp ? p[4 * NR + 3 * NS + k] : 0.0;
      L.cv1[m] = sp ? p[4 * NR + 4 * NS + k] : 0.0;
    }}
    L.rho = g[i];
    L.irho = 1.0 / L.rho;
    L.bnd = kBnd[x.r];
    // the zero that pads the term sequences
    if (x.r == 0) x.lds[kOffQ + kSentinel] = 0.0;
  }}
}};

}}  // namespace gen_{tag}
}}  // namespace rkmi
"""
    source = f"""// Generated by paper_1611_02274_amd/codegen.py -- do not edit.
// Launchers of the {n}-species network with the energy equation (topology {tag}): the
// group kernels under every schedule; no host build of the per-system code.
#include "net_{tag}.hpp"

extern "C" int rkmi_gen_{tag}_launch(const rkmi::LaunchArgs* a, void* s) {{
  return rkmi::launch_group_only<rkmi::gen_{tag}::GNet>(a, s);
}}

extern "C" int rkmi_gen_{tag}_host(const rkmi::LaunchArgs*) {{
  return rkmi::kLaunchInvalid;
}}

extern "C" int64_t rkmi_gen_{tag}_workspace(int, int, int64_t n) {{
  return n > 0 ? (int64_t)rkmi::kQueueBytes : 0;
}}
"""
    return header, source


def _species_terms(net):
    """Per species, the signed rates of its omega sum in evaluation order:
    reaction by reaction, reactant slots (subtract) before product slots (add).
    Entries are q_index << 1 | negative."""
    terms = [[] for _ in range(net.n_sp)]
    for j in range(net.n_rx):
        for k in net.reac[j]:
            if k >= 0:
                terms[int(k)].append(j << 1 | 1)
        for k in net.prod[j]:
            if k >= 0:
                terms[int(k)].append(j << 1)
    return terms


def _table(name, ctype, values, per_line=16, align=0):
    rows = [", ".join(str(v) for v in values[i:i + per_line])
            for i in range(0, len(values), per_line)]
    body = ",\n      ".join(rows)
    al = f"alignas({align}) " if align else ""
    return f"  {al}static constexpr {ctype} {name}[{len(values)}] = {{\n      {body}}};"


# Group variants: a lane's species list is consumed in chunks of this many
# terms; its first species' list is padded to a whole number of chunks.
GROUP_TERM_CHUNK = 4
# doubles of the group scratch that hold the RKC stage recurrence (RkcCoef, 11
# doubles) between evaluations for stage counts above the tabulated ones
GROUP_COEF_DOUBLES = 12


def _group_positions(net, L, R):
    """Reaction -> rate position p = m * L + r (slot m of lane r).  Reactions
    with a one-species side (times [M]) fill the last slots, so the kernel
    selects [M] for an operand only there; the others fill the first slots in
    reaction order.  Returns (position of each reaction, reaction of each
    position or -1, first slot that may hold a [M] reaction)."""
    nr, n = net.n_rx, net.n_sp
    third = [j for j in range(nr) if int(net.reac[j][1]) < 0 or int(net.prod[j][1]) < 0]
    plain = [j for j in range(nr) if j not in set(third)]
    m_slots = -(-len(third) // L) if third else 0
    # the [M] slots also take the plain reactions that do not fit before them
    m_first = R - m_slots
    while m_first > 0 and len(plain) > m_first * L:
        m_first -= 1
    front = plain[:m_first * L]
    back = plain[m_first * L:] + third
    assert len(back) <= (R - m_first) * L
    pos_of = [-1] * nr
    rx_of = [-1] * (R * L)
    for p, j in enumerate(front):
        pos_of[j], rx_of[p] = p, j
    for t, j in enumerate(back):
        p = m_first * L + t
        pos_of[j], rx_of[p] = p, j
    return pos_of, rx_of, (m_first if third else R)


def _group_species(lens, L, chunk):
    """Species -> (lane, slot) for two slots per lane: each lane sums its
    slot-0 species' terms (padded to whole chunks), then its slot-1 species'.
    The heaviest lists go alone to a lane (in slot 1: no padding); the rest
    are paired heavy with light, each pair ordered for the shorter padded
    sequence.  Returns sp[slot * L + lane] (-1: none)."""
    n = len(lens)
    assert L < n <= 2 * L
    order = sorted(range(n), key=lambda k: (-lens[k], k))
    single = 2 * L - n
    sp = [-1] * (2 * L)
    for r in range(single):
        sp[L + r] = order[r]
    rest = order[single:]
    m = len(rest)

    def padded(k):
        return -(-lens[k] // chunk) * chunk

    for i in range(m // 2):
        a, b = rest[i], rest[m - 1 - i]
        if padded(b) + lens[a] < padded(a) + lens[b]:
            a, b = b, a
        sp[single + i] = a
        sp[L + single + i] = b
    return sp


def _group_layout(net, L, thermal=False):
    """The group layout of a network (rk_group.hpp): reaction positions,
    operand codes, the unknowns of each lane's slots (isothermal: species k
    is unknown k; with the energy equation T is unknown 0 and species k is
    unknown 1 + k), the LDS area and each lane's packed term sequence."""
    n, nr = net.n_sp, net.n_rx
    nu = n + 1 if thermal else n          # unknowns
    S, R = -(-nu // L), -(-nr // L)
    assert S == 2, "group variants hold two unknowns per lane"
    assert n < 255, "species indices are packed in bytes"
    chunk = GROUP_TERM_CHUNK
    pos_of, rx_of, m_first = _group_positions(net, L, R)
    rx = []
    for p in range(R * L):
        j = rx_of[p]
        if j >= 0:
            a, b = int(net.reac[j][0]), int(net.reac[j][1])
            c, d = int(net.prod[j][0]), int(net.prod[j][1])
            b = n if b < 0 else b
            d = n if d < 0 else d
            rx.append(a | b << 8 | c << 16 | d << 24)
        else:
            rx.append(0)
    # LDS area of a system (doubles): C [0, NS] (C_N the [M] operand's place;
    # with the energy equation T at NS + 1) | rates +q at kOffQ + p, p < R*L,
    # the zero at kOffQ + R*L, scratch (16-byte aligned: the norms over the
    # unknowns; with the energy equation also two species sums) | -q at
    # kOffQ + kNegOff + p
    c_len = n + (2 if thermal else 1)
    off_q = c_len + c_len % 2
    off_red = off_q + R * L + 1 + (off_q + R * L + 1) % 2
    # with the energy equation the two species rows follow the RKC recurrence's
    # coefficients, which stay in the scratch across evaluations
    off_e1 = off_red + GROUP_COEF_DOUBLES
    off_e2 = off_e1 + n + n % 2
    red_len = max(nu, off_e2 + n + n % 2 - off_red) if thermal else nu
    neg = off_red - off_q + red_len
    lds_per_system = off_q + neg + R * L
    lds_per_system += lds_per_system % 2
    sentinel = R * L
    sterms = [[pos_of[c >> 1] + neg * (c & 1) for c in lst] for lst in _species_terms(net)]
    terms = ([[]] + sterms) if thermal else sterms     # per unknown
    lens = [len(t) for t in terms]
    sp = _group_species(lens, L, chunk)
    seqs, bnd = [], []
    for r in range(L):
        k0, k1 = sp[r], sp[L + r]
        l0 = terms[k0] if k0 >= 0 else []
        l0 = l0 + [sentinel] * ((-len(l0)) % chunk)
        l1 = terms[k1] if k1 >= 0 else []
        seqs.append(l0 + l1)
        bnd.append(len(l0) // chunk)
    tot = max(len(q) for q in seqs)
    tot += (-tot) % chunk
    assert tot // chunk <= 64
    seqs = [q + [sentinel] * (tot - len(q)) for q in seqs]
    bits = (neg + R * L).bit_length()
    per_word = 32 // bits
    n_words = max(1, -(-tot // per_word))
    tc = [0] * (n_words * L)
    for r in range(L):
        for t, code in enumerate(seqs[r]):
            tc[(t // per_word) * L + r] |= code << ((t % per_word) * bits)
    return dict(n=n, nr=nr, nu=nu, L=L, S=S, R=R, m_first=m_first, rx=rx, rx_of=rx_of,
                off_q=off_q, off_red=off_red, off_e1=off_e1, off_e2=off_e2, neg=neg,
                lds_per_system=lds_per_system,
                sentinel=sentinel, sp=sp, bnd=bnd, tot=tot, bits=bits, per_word=per_word,
                n_words=n_words, tc=tc, chunk=chunk,
                switch=sum(1 << (b - 1) for b in set(bnd) if b > 0))


def _lane_major(words, L, per_lane):
    """A [per_lane][L] table (entry w of lane r at w L + r) as [L][per_lane']
    with per_lane' = per_lane rounded up to whole 16-byte vectors (zeros)."""
    padded = -(-per_lane // 4) * 4
    out = [0] * (L * padded)
    for r in range(L):
        for w in range(per_lane):
            out[r * padded + w] = words[w * L + r]
    return out, padded


def _group_tables(G) -> str:
    rx, rx_words = _lane_major(G["rx"], G["L"], G["R"])
    tc, tc_words = _lane_major(G["tc"], G["L"], G["n_words"])
    return f"""{_table("kSp", "int", G["sp"])}
{_table("kRxOf", "int16_t", G["rx_of"])}
  // lane r's operand codes and packed term codes, each lane's contiguous and
  // 16-byte aligned (read as whole vectors at every evaluation)
  static constexpr int kRxWords = {rx_words};
  static constexpr int kTcWords = {tc_words};
{_table("kRx", "uint32_t", rx, align=16)}
{_table("kTc", "uint32_t", tc, align=16)}
{_table("kBnd", "int", G["bnd"])}
  // chunks at whose end some lane moves its accumulator to slot 0 (bit c)
  static constexpr uint64_t kSwitchChunks = {G["switch"]}ull;"""


def group_source(net, tag: str, lanes: int | None = None) -> str:
    """The group variant of a network (kernels of rk_group.hpp): lane r of a
    group of `lanes` computes the rates of progress at its positions
    p = m*lanes + r (_group_positions) and owns the species of its two slots
    (_group_species); per lane: the species of each slot, the packed operand
    species of each position's reaction, and the signed rate positions of its
    species' sums in reaction order (slot 0's list, padded to whole chunks,
    then slot 1's), packed into registers."""
    n, nr = net.n_sp, net.n_rx
    L = lanes or group_lanes(n)
    G = _group_layout(net, L)
    S, R, m_first = G["S"], G["R"], G["m_first"]
    off_q, sentinel, neg, off_red = G["off_q"], G["sentinel"], G["neg"], G["off_red"]
    lds_per_system, bits, per_word, n_words = (G["lds_per_system"], G["bits"], G["per_word"],
                                               G["n_words"])
    tot, chunk = G["tot"], G["chunk"]
    return f"""
// Group variant: {L} lanes per system (rk_group.hpp).
struct GNet {{
  static constexpr int N = {n};
  static constexpr int NR = {nr};
  static constexpr int kL = {L};
  static constexpr int kGroupLanes = {L};
  static constexpr bool kColumns = false;
  static constexpr int kLaneDoubles = 0;
  // three waves per SIMD: the evaluation loop fits 168 registers (the power
  // method and the set-up of a system run out of line)
  static constexpr int kWavesPerEuRkc = 2;
  static constexpr int kWavesPerEuRkck = 3;
  static constexpr int S = {S};
  static constexpr int R = {R};
  static constexpr int kMSlot = {m_first};   // first slot that may hold a [M] reaction
  static constexpr int kOffC = 0;
  static constexpr int kOffQ = {off_q};
  static constexpr int kSentinel = {sentinel};
  static constexpr int kNegOff = {neg};
  static constexpr int kOffRed = {off_red};
  static constexpr int kLdsPerSystem = {lds_per_system};
  static constexpr int kTermBits = {bits};
  static constexpr int kTermsPerWord = {per_word};
  static constexpr int kTermWords = {n_words};
  static constexpr int kTermLen = {tot};
  static constexpr int kChunk = {chunk};
  using Params = const double*;
{_group_tables(G)}
  struct Lane {{
    double kf[R], kr[R];
    double W[S], iW[S];
    double rho, irho;
    int bnd;   // chunks of the slot-0 list
  }};
  // The forward rate constants of a lane's positions into the group's rate
  // area; once per system, out of line (the exponentials' temporaries do not
  // count against the registers of the evaluation loop).
  __device__ __attribute__((noinline)) static void rates(Params p, double T, double* lds, int r) {{
    const double lnT = crm::cr_log(T);
    double* const Q = lds + kOffQ;
#pragma nounroll
    for (int m = 0; m < R; ++m) {{
      const int j = kRxOf[m * kL + r];
      if (j >= 0) Q[m * kL + r] = crm::cr_exp(p[j] + p[NR + j] * lnT - p[2 * NR + j] / T);
    }}
  }}
  __device__ static void init(Lane& L, const Params& p, const double* __restrict__ g, int64_t i,
                              int64_t n, const Grp<GNet>& x) {{
    const double T = g[i];
    const double rho = g[n + i];
    double* const Q = x.lds + kOffQ;
    rates(p, T, x.lds, x.r);
#pragma unroll
    for (int m = 0; m < R; ++m) {{
      const int j = kRxOf[m * kL + x.r];
      L.kf[m] = j >= 0 ? Q[m * kL + x.r] : 0.0;
      L.kr[m] = j >= 0 ? L.kf[m] * p[3 * NR + j] : 0.0;
    }}
#pragma unroll
    for (int m = 0; m < S; ++m) {{
      const int k = x.sp[m];
      L.W[m] = k >= 0 ? p[4 * NR + k] : 0.0;
      L.iW[m] = k >= 0 ? p[4 * NR + N + k] : 0.0;
    }}
    L.rho = rho;
    L.irho = 1.0 / rho;
    L.bnd = kBnd[x.r];
    if (x.r == 0) Q[kSentinel] = 0.0;
  }}
}};
"""


def _vjp_source(net) -> str:
    """Vector-Jacobian products of the rate law, for the discrete adjoint:
    jtu = J(y)^T u and th += (df/dlnA)^T u.  With u~_k = (W_k / rho) u_k and
    r_j = sum_k nu_kj u~_k, both rate constants scale with A_j, so
    d(u^T f)/dlnA_j = r_j q_j; the concentrations take the adjoints of the
    products, [M] the adjoints of its factors, and (J^T u)_k =
    (rho / W_k) (C^_k + [M]^).  Same operations, same order, as the reference
    evaluation (products left to right, accumulators from zero)."""
    lines = []
    for j in range(net.n_rx):
        a, b = int(net.reac[j][0]), int(net.reac[j][1])
        c, d = int(net.prod[j][0]), int(net.prod[j][1])
        x = f"-uw[{b}]" if b >= 0 else "0.0"
        y = f"uw[{d}]" if d >= 0 else "0.0"
        lines.append(f"    r = ((-uw[{a}] + {x}) + uw[{c}]) + {y};")
        lines.append(f"    kf = L.kf[z + {j} * kLdsStride];")
        lines.append(f"    kr = kf * ld_uniform(iK, {j});")
        lines.append(f"    th[{j}] += r * ({_side('kf', net.reac[j])} - {_side('kr', net.prod[j])});")
        lines.append("    t = r * kf;")
        if b >= 0:
            lines.append(f"    Cb[{a}] += t * C[{b}];")
            lines.append(f"    Cb[{b}] += t * C[{a}];")
        else:
            lines.append(f"    Cb[{a}] += t * M;")
            lines.append(f"    Mb += t * C[{a}];")
        lines.append("    t = -r * kr;")
        if d >= 0:
            lines.append(f"    Cb[{c}] += t * C[{d}];")
            lines.append(f"    Cb[{d}] += t * C[{c}];")
        else:
            lines.append(f"    Cb[{c}] += t * M;")
            lines.append(f"    Mb += t * C[{c}];")
    body = "\n".join(lines)
    return f"""  static constexpr int kNTheta = NR;
  template <class VI, class VU, class VO>
  RKMI_HD static void vjp(const Lane& L, const Params& p, const VI& y, const VU& u, VO& jtu,
                          double (&th)[NR]) {{
    const double* __restrict__ iK = p + 3 * NR;
    const double* __restrict__ W = p + 4 * NR;
    const double* __restrict__ iW = W + N;
    double C[N], uw[N], Cb[N];
    const int z = opaque_zero();
#pragma unroll
    for (int k = 0; k < N; ++k) C[k] = (L.rho * y[k]) * ld_uniform(iW, k);
    double M = 0.0;
#pragma unroll
    for (int k = 0; k < N; ++k) M += C[k];
#pragma unroll
    for (int k = 0; k < N; ++k) uw[k] = (ld_uniform(W, k) * L.irho) * u[k];
#pragma unroll
    for (int k = 0; k < N; ++k) Cb[k] = 0.0;
    double Mb = 0.0;
    double r, kf, kr, t;
{body}
#pragma unroll
    for (int k = 0; k < N; ++k) jtu[k] = (L.rho * ld_uniform(iW, k)) * (Cb[k] + Mb);
  }}
"""


def _adjoint_exports(tag) -> str:
    return f"""
extern "C" int rkmi_gen_{tag}_taped(const rkmi::LaunchArgs* a, const rkmi::TapeArgs* t, void* s) {{
  return rkmi::launch_taped<rkmi::gen_{tag}::Net>(a, t, s);
}}

extern "C" int rkmi_gen_{tag}_taped_host(const rkmi::LaunchArgs* a, const rkmi::TapeArgs* t) {{
  return rkmi::host_taped<rkmi::gen_{tag}::Net>(a, t);
}}

extern "C" int rkmi_gen_{tag}_adjoint(const rkmi::AdjointArgs* a, void* s) {{
  return rkmi::launch_adjoint<rkmi::gen_{tag}::Net>(a, s);
}}

extern "C" int rkmi_gen_{tag}_adjoint_host(const rkmi::AdjointArgs* a) {{
  return rkmi::host_adjoint<rkmi::gen_{tag}::Net>(a);
}}
"""


def batch_source(tags, key: str) -> str:
    """One translation unit with the ragged-batch kernels over the networks
    `tags` (in this order)."""
    inc = "\n".join(f'#include "net_{t}.hpp"' for t in tags)
    nets = ", ".join(f"rkmi::gen_{t}::Net" for t in tags)
    return f"""// Generated by paper_1611_02274_amd/codegen.py -- do not edit.
// Ragged batch over {len(tags)} networks: {", ".join(tags)}.
{inc}
#include "../rk_batch.hpp"

extern "C" int rkmi_batch_{key}_launch(const rkmi::BatchArgs* a, void* s) {{
  return rkmi::batch_launch<{nets}>(a, s);
}}

extern "C" int64_t rkmi_batch_{key}_workspace(const rkmi::BatchArgs* a) {{
  return rkmi::batch_workspace<{nets}>(a);
}}

extern "C" void rkmi_batch_{key}_free(void* cache) {{ rkmi::batch_free_cache(cache); }}
"""


def batch_key(tags) -> str:
    import hashlib
    return hashlib.sha1("/".join(tags).encode()).hexdigest()[:8]


def registry_source(entries, batches=(), thermal=()) -> str:
    """entries: list of (tag, net); batches: lists of tags compiled together;
    thermal: list of (tag, net) compiled with the energy equation."""
    decl, tabs, rows = [], [], []
    for tag, net in thermal:
        decl.append(f'extern "C" int rkmi_gen_{tag}_launch(const rkmi::LaunchArgs*, void*);')
        decl.append(f'extern "C" int rkmi_gen_{tag}_host(const rkmi::LaunchArgs*);')
        decl.append(f'extern "C" int64_t rkmi_gen_{tag}_workspace(int, int, int64_t);')
    for tag, net in entries:
        decl.append(f'extern "C" int rkmi_gen_{tag}_launch(const rkmi::LaunchArgs*, void*);')
        decl.append(f'extern "C" int rkmi_gen_{tag}_host(const rkmi::LaunchArgs*);')
        decl.append(f'extern "C" int64_t rkmi_gen_{tag}_workspace(int, int, int64_t);')
        if net.n_sp <= REGISTER_SPECIES_LIMIT:
            decl.append(f'extern "C" int rkmi_gen_{tag}_taped(const rkmi::LaunchArgs*, '
                        'const rkmi::TapeArgs*, void*);')
            decl.append(f'extern "C" int rkmi_gen_{tag}_taped_host(const rkmi::LaunchArgs*, '
                        'const rkmi::TapeArgs*);')
            decl.append(f'extern "C" int rkmi_gen_{tag}_adjoint(const rkmi::AdjointArgs*, void*);')
            decl.append(f'extern "C" int rkmi_gen_{tag}_adjoint_host(const rkmi::AdjointArgs*);')
            adj = (f"rkmi_gen_{tag}_taped, rkmi_gen_{tag}_taped_host, rkmi_gen_{tag}_adjoint, "
                   f"rkmi_gen_{tag}_adjoint_host")
        else:
            adj = "nullptr, nullptr, nullptr, nullptr"
        r = ", ".join(str(int(x)) for x in np.asarray(net.reac).reshape(-1))
        p = ", ".join(str(int(x)) for x in np.asarray(net.prod).reshape(-1))
        tabs.append(f"static const int32_t reac_{tag}[] = {{{r}}};")
        tabs.append(f"static const int32_t prod_{tag}[] = {{{p}}};")
        rows.append(f"    {{{net.n_sp}, {net.n_rx}, reac_{tag}, prod_{tag}, rkmi_gen_{tag}_launch, "
                    f"rkmi_gen_{tag}_host, rkmi_gen_{tag}_workspace, {adj}, 0}},")
    index = {tag: k for k, (tag, _) in enumerate(entries)}
    for tag, net in thermal:
        base = tag[:-len(THERMAL_SUFFIX)]
        if f"static const int32_t reac_{base}[]" not in "\n".join(tabs):
            r = ", ".join(str(int(x)) for x in np.asarray(net.reac).reshape(-1))
            p = ", ".join(str(int(x)) for x in np.asarray(net.prod).reshape(-1))
            tabs.append(f"static const int32_t reac_{base}[] = {{{r}}};")
            tabs.append(f"static const int32_t prod_{base}[] = {{{p}}};")
        rows.append(f"    {{{net.n_sp}, {net.n_rx}, reac_{base}, prod_{base}, rkmi_gen_{tag}_launch, "
                    f"rkmi_gen_{tag}_host, rkmi_gen_{tag}_workspace, "
                    "nullptr, nullptr, nullptr, nullptr, 1},")
    brows = []
    for tags in batches:
        key = batch_key(tags)
        decl.append(f'extern "C" int rkmi_batch_{key}_launch(const rkmi::BatchArgs*, void*);')
        decl.append(f'extern "C" int64_t rkmi_batch_{key}_workspace(const rkmi::BatchArgs*);')
        decl.append(f'extern "C" void rkmi_batch_{key}_free(void*);')
        idx = ", ".join(str(index[t]) for t in tags)
        brows.append(f"    {{{len(tags)}, {{{idx}}}, rkmi_batch_{key}_launch, "
                     f"rkmi_batch_{key}_workspace, rkmi_batch_{key}_free}},")
    if not brows:
        brows.append("    {0, {0}, nullptr, nullptr, nullptr},")
    return (
        "// Generated by paper_1611_02274_amd/codegen.py -- do not edit.\n"
        "// Networks compiled into the library, matched by exact topology.\n"
        '#include "../rk_types.hpp"\n\n' + "\n".join(decl) + "\n\n" + "\n".join(tabs) +
        "\n\nnamespace rkmi {\nextern const GenEntry kGenRegistry[] = {\n" + "\n".join(rows) +
        "\n};\nextern const int kGenRegistrySize = " + str(len(rows)) + ";\n" +
        "extern const BatchEntry kBatchRegistry[] = {\n" + "\n".join(brows) + "\n};\n" +
        "extern const int kBatchRegistrySize = " + str(len(batches)) + ";\n"
        "}  // namespace rkmi\n")


def tag_of(net) -> str:
    return f"n{net.n_sp}r{net.n_rx}_{net.topology_key()[:8]}"


THERMAL_SUFFIX = "_th"


def generate(nets, out_dir: str = GEN_DIR, batches=(), thermal=()) -> list[str]:
    """Writes one source per network, one per batch (lists of networks compiled
    together), one per network compiled with the energy equation (`thermal`)
    and the registry; returns the paths of the sources to compile.  Files
    whose content is unchanged are left untouched."""
    os.makedirs(out_dir, exist_ok=True)
    paths, entries, tentries = [], [], []
    keep = set()
    for net in thermal:
        tag = tag_of(net) + THERMAL_SUFFIX
        tentries.append((tag, net))
        header, source = (thermal_source(net, tag) if net.n_sp + 1 <= REGISTER_SPECIES_LIMIT
                          else thermal_group_source(net, tag))
        keep.add(os.path.basename(_write(os.path.join(out_dir, f"net_{tag}.hpp"), header)))
        paths.append(_write(os.path.join(out_dir, f"net_{tag}.hip"), source))
    for net in nets:
        tag = tag_of(net)
        entries.append((tag, net))
        header, source = rhs_source(net, tag)
        keep.add(os.path.basename(_write(os.path.join(out_dir, f"net_{tag}.hpp"), header)))
        paths.append(_write(os.path.join(out_dir, f"net_{tag}.hip"), source))
    btags = [[tag_of(n) for n in b] for b in batches]
    for tags in btags:
        paths.append(_write(os.path.join(out_dir, f"batch_{batch_key(tags)}.hip"),
                            batch_source(tags, batch_key(tags))))
    paths.append(_write(os.path.join(out_dir, "registry.cpp"),
                        registry_source(entries, btags, tentries)))
    keep |= {os.path.basename(p) for p in paths}
    for f in os.listdir(out_dir):
        if f not in keep and f.startswith(("net_", "registry.", "batch_")):
            os.remove(os.path.join(out_dir, f))
    return paths


def _write(path: str, text: str) -> str:
    if os.path.exists(path):
        with open(path) as fh:
            if fh.read() == text:
                return path
    with open(path, "w") as fh:
        fh.write(text)
    return path


def standard_nets():
    from .inputs import standard_network
    return [standard_network(k) for k in (9, 13, 32, 53)]
