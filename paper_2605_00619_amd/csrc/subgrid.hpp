// Host construction of the sub-tetrahedral grid, the agglomerated cell DOFs
// and the boundary-triangle pairing of a periodic or bounded polyhedral mesh.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/afe.h"

namespace afe {

struct HostGrid {
    int N = 0, np = 0, nf = 0;
    int n_cells = 0;
    int64_t ndof = 0, nsub = 0;
    int max_cell_dofs = 0, max_cell_subtets = 0;
    double box = 1.0, h_min = 0.0;
    std::vector<int64_t> dof_ptr;   // [n_cells + 1]
    std::vector<int64_t> sub_ptr;   // [n_cells + 1]
    std::vector<int32_t> conn;      // [nsub][np] cell-local DOF
    std::vector<int32_t> sub_cell;  // [nsub]
    std::vector<double> geo;        // [nsub][10]: G = J^{-1} row-major (9), |det J|
    std::vector<double> tri;        // [nsub][4]: 2 * area, unit normal (outward)
    std::vector<int32_t> nbr_sub;   // [nsub] neighbour's sub-tet on the same triangle; -1 - b on
                                    // boundary triangle b of a bounded mesh
    int64_t n_btri = 0;             // boundary triangles (bounded meshes)
    std::vector<double> bnode_x;    // [n_btri][nf][3] coordinates of their face nodes
    std::vector<int32_t> perm;      // [nsub][nf] matching face node in the neighbour
    std::vector<double> h, vol;     // [n_cells] diameter, volume
    std::vector<double> mrow;       // [ndof] int_P phi_l (column sums of M_i)
    std::vector<double> dof_x;      // [3][ndof] DOF coordinates, cell frame
    std::vector<int32_t> dof_cell;  // [ndof]
    std::vector<int32_t> inc_ptr, inc_idx;    // DOF -> (sub-tet*np + node), ascending
    std::vector<int32_t> finc_ptr, finc_idx;  // DOF -> (sub-tet*nf + face node), ascending
};

// Returns AFE_OK or an error code with a message in `err`.
afe_status build_host_grid(const afe_mesh &mesh, int N, HostGrid &g, std::string &err);

}  // namespace afe
