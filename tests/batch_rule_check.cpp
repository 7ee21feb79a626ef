// Prints batch_rule(avail, per, want) for each "avail per want" line on stdin
// (tests/test_host_tables.py checks the documented rule on the output).
#include <cstdio>

#include "batch_rule.h"

int main() {
    unsigned long long avail, per;
    int want;
    while (std::scanf("%llu %llu %d", &avail, &per, &want) == 3)
        std::printf("%d\n", dfl::batch_rule((size_t)avail, (size_t)per, want));
    return 0;
}
