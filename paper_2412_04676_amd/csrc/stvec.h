// Start vector of the next two-site position from the split of the current one.
#pragma once
#include "hpsi.h"

namespace bsd {

// psi: wave function at (site, site+1) in its layout; the site tensor of `site`
// (left_to_right) or of site+1 (right to left) must already hold the kept
// singular vectors.  guess receives the start vector at site+1 (site-1) in the
// layout of that position, whose environment blocks must exist.  work is
// scratch for the intermediate blocks.  Synchronizes s.
void next_guess(Ctx& ctx, int site, bool left_to_right, const double* psi, double* guess, DevBuf& work,
                hipStream_t s);

}  // namespace bsd
