// Internal declarations shared by the host structure builder and the HIP
// part of the library.  Not part of the public ABI.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/pmcorr.h"

namespace pm {

// Everything about a mesh that does not depend on material parameters.
// Per-side arrays are [cell][3] in the caller's cell order.
struct HostStructure {
  int32_t n_nodes = 0;
  int32_t n = 0;                 // cells
  std::vector<int32_t> nbr;      // neighbour across side j, or -1
  std::vector<int32_t> nbr_side; // side index in the neighbour, or -1
  std::vector<double> cot;       // cot of the angle opposite side j
  std::vector<double> T;         // l/d (interior) or l/delta_b (boundary, 0 if cot <= 0)
  std::vector<double> tx, ty;    // side vector, node j+1 -> node j+2
  std::vector<double> area;      // per cell
  std::vector<int8_t> tag;       // Dirichlet bit mask on boundary sides, 0 on interior sides
  std::vector<int32_t> perm;     // perm[new] = old
  std::vector<int32_t> inv;      // inv[old] = new
  std::vector<int32_t> row_ptr;  // CSR in the new order
  std::vector<int32_t> col;
  std::vector<int32_t> comp;     // connected component of each cell
  std::vector<uint8_t> comp_bits;  // OR of the Dirichlet bits present in each component
  pm_mesh_stats stats{};
};

// Validates the mesh and fills hs; returns a PM_* status and a message.
int build_structure(int32_t n_nodes, const double* xy, int32_t n_cells, const int32_t* tri,
                    const int8_t* side_tag, HostStructure& hs, std::string& err);

// Host structure of a mesh handle (defined with pm_mesh).
const HostStructure* mesh_structure(const pm_mesh* m);

// Thread-local last error message (set by the C entry points).
void set_error(int status, const std::string& msg);

}  // namespace pm
