// Locally corrected near-field quadrature (paper section 2.2).
#include "plan.hpp"

namespace fdbem {

void build_corrections(Plan &P)
{
    P.has_corr = false;
}

}  // namespace fdbem
