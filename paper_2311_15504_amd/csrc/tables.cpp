// Host copies of the compile-time ENO-MR coefficient table.
#include "tables.hpp"

namespace enomr {

bool generate_tables(double a[kPool][kMaxW], double b[kPool][kMaxW])
{
    for (int c = 0; c < kPool; ++c)
        for (int l = 0; l < kMaxW; ++l) {
            a[c][l] = kCoef.a[c][l];
            b[c][l] = kCoef.b[c][l];
        }
    return true;
}

}  // namespace enomr
