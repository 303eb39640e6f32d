"""Host logic of the Newton-pair split of the FP32 field (sym_split and its
helpers in ct_internal.hpp), compiled for the host: Eq. 4 is antisymmetric,
so the split may evaluate each unordered pair of holes once, and it must then
meet every unordered pair of tiles exactly once (offset 0: each tile with
itself), send every reaction to a partial slot inside the event's allocation,
and make each tile wait for exactly the contributions it receives.  Checked
by brute force over tile counts and chunk lengths; past the tile limit the
items are one-sided and at most kMaxChunks per tile."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2506_09712_amd", "csrc")
HIPCC = "/opt/rocm/bin/hipcc"

PROGRAM = r"""
#include "ct_internal.hpp"
#include <algorithm>
#include <cstdio>
#include <vector>

static int check(int T, int C)
{
    const int n = T * ct::kSymTile - (T > 1 ? 17 : 0);  // a ragged last tile
    const ct::SymSplit s = ct::sym_split(n, C);
    if (s.T != T || !s.newton) return 1;
    std::vector<int> met((size_t)T * T, 0), recv(T, 0);
    for (int a = 0; a < T; ++a) {
        const int pa = ct::sym_partners(T, a);
        if (pa > s.P || (pa + s.C - 1) / s.C > s.R) return 2;
        for (int r = 0; r < s.R; ++r)
            for (int o = r * s.C; o < std::min(r * s.C + s.C, pa); ++o) {
                if (o == 0) continue;
                const int b = (a + o) % T;
                if (b == a) return 3;
                met[(size_t)std::min(a, b) * T + std::max(a, b)] += 1;
                recv[b] += 1;
                if (s.R + o - 1 >= ct::sym_slots(s)) return 4;  // reaction slot
            }
        if (T > 1 && s.R > ct::sym_slots(s)) return 5;  // own slots
    }
    for (int a = 0; a < T; ++a)
        for (int b = a + 1; b < T; ++b)
            if (met[(size_t)a * T + b] != 1) return 6;
    for (int b = 0; b < T; ++b) {
        if (recv[b] != ct::sym_received(T, b)) return 7;
        if (ct::sym_expected(s, b) != s.R + recv[b]) return 8;
    }
    if (ct::sym_partials(s) != (T > 1)) return 9;
    return 0;
}

int main()
{
    for (int C = 1; C <= ct::kSymMaxC; ++C) {
        for (int T = 1; T <= 160; ++T)
            if (int e = check(T, C)) { std::printf("T %d C %d: %d\n", T, C, e); return 1; }
        for (int T : {255, 256, 511, 512})
            if (int e = check(T, C)) { std::printf("T %d C %d: %d\n", T, C, e); return 1; }
    }
    for (int T : {513, 600, 5000, 70000})
        for (int C : {1, 5, 15}) {
            const ct::SymSplit s = ct::sym_split(T * ct::kSymTile, C);
            if (s.newton || s.R > ct::kMaxChunks || (long)s.R * s.C < T || s.C < C ||
                ct::sym_expected(s, 0) != s.R || !ct::sym_partials(s)) {
                std::printf("one-sided T %d C %d\n", T, C);
                return 1;
            }
        }
    std::puts("split ok");
    return 0;
}
"""


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc is not installed")
def test_newton_split_meets_every_pair_once(tmp_path):
    src = tmp_path / "split.hip"
    src.write_text(PROGRAM)
    exe = tmp_path / "split"
    subprocess.run([HIPCC, "-std=c++17", "-O2", "--offload-arch=gfx950", "-I", CSRC,
                    "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True, capture_output=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and "split ok" in r.stdout, r.stdout + r.stderr


ORDER_PROGRAM = r"""
#include "ct_internal.hpp"
#include <cstdio>
#include <vector>

// deposit_major must be a bijection of [0, n) whose slots run deposit by
// deposit (carrier k on deposit k mod nd), each deposit's carriers in
// increasing order.
int main()
{
    for (int nd : {0, 1, 2, 3, 7, 40, 41, 100})
        for (int n : {0, 1, 2, 5, 39, 40, 41, 79, 80, 81, 1389, 55556, 55557}) {
            std::vector<int> seen(n > 0 ? n : 1, 0);
            int prev_d = -1, prev_k = -1;
            for (int s = 0; s < n; ++s) {
                const int k = ct::deposit_major(s, n, nd);
                if (k < 0 || k >= n || seen[k]++) { std::printf("nd %d n %d s %d: k %d\n", nd, n, s, k); return 1; }
                if (nd <= 1) { if (k != s) return 2; continue; }
                const int d = k % nd;
                if (d < prev_d || (d == prev_d && k <= prev_k)) { std::printf("order nd %d n %d s %d\n", nd, n, s); return 3; }
                prev_d = d;
                prev_k = k;
            }
        }
    std::puts("order ok");
    return 0;
}
"""


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc is not installed")
def test_deposit_major_slot_order_is_a_bijection(tmp_path):
    src = tmp_path / "order.hip"
    src.write_text(ORDER_PROGRAM)
    exe = tmp_path / "order"
    subprocess.run([HIPCC, "-std=c++17", "-O2", "--offload-arch=gfx950", "-I", CSRC,
                    "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True, capture_output=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and "order ok" in r.stdout, r.stdout + r.stderr
