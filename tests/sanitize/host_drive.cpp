// host_drive.cpp -- exercises the library's host-side operator construction
// (translation tables of both expansion families, the same-level M2L plan,
// the BF16 split, general M2L operators) for every supported order, so that
// a build with AddressSanitizer and UndefinedBehaviorSanitizer can report
// out-of-bounds accesses, overflow and the like.  Test infrastructure;
// prints "ok" when done.
#include <cmath>
#include <cstdio>
#include <cstdlib>

#include "host_ops.h"

int main() {
    using namespace fmm;
    for (int p = 0; p <= 16; p++) {
        HostTables t;
        build_tables(p, t);
        if (t.K != (p + 1) * (p + 1) || t.KP != kpad(p)) return 1;
        std::vector<double> op;
        const double q[3] = {2.0, -1.0, 3.0};
        m2l_operator(p, q, 0.5, op);
        if (op.size() != (size_t)t.K * t.K) return 2;
        for (double v : op)
            if (!std::isfinite(v)) return 3;
    }
    for (int p = 0; p <= 6; p++) {
        HostTables t;
        build_tables_cart(p, t);
        if (t.K != (p + 1) * (p + 2) * (p + 3) / 6 || t.KP != kpad_cart(p)) return 4;
    }
    const double thetas[] = {0.7, 0.5, 0.4};
    for (double th : thetas) {
        for (int p : {1, 4, 8}) {
            M2LPlan plan;
            build_m2l_plan(p, th, plan);
            if (plan.J != m2l_plan_slots(th)) return 5;
            std::vector<uint16_t> hi, lo;
            const int KP = kpad(p);
            split_bf16_kblocked(plan.T, plan.offsets.size(), KP, hi, lo);
            if (hi.size() != plan.T.size() || lo.size() != plan.T.size()) return 6;
        }
        M2LPlan pc;
        build_m2l_plan(4, th, pc, true);
        if (pc.J != m2l_plan_slots(th)) return 7;
    }
    // slot counts only, down to the smallest opening angle the traversal accepts
    for (double th = 0.95; th > 0.05; th *= 0.8)
        if (m2l_plan_slots(th) < 0) return 8;
    std::printf("ok\n");
    return 0;
}
