#pragma once
#include <vector>

namespace tdse {

// The `count` lowest eigenpairs of the field-free radial block h_l on the grid
// r_i = (i+1) dr (stencil 3 or 5, zero padding).  energies[k]; vectors[k*n + i]
// normalised to dr * sum phi^2 = 1, largest component positive.
void lowest_radial_states(int n, int stencil, double dr, double z, int l, int count,
                          std::vector<double>& energies, std::vector<double>& vectors);

}  // namespace tdse
