// Host tables of a mesh with one degree per cell (built once per problem).
#pragma once

#include <cstdint>
#include <vector>

#include "hpg_internal.h"
#include "kernels.h"

namespace hpg {

struct HpHost {
    std::vector<RefTables> ref;             // by degree (2..pmax)
    std::vector<double> tab;                // packed reference tables
    std::vector<dev::HpTabOff> toff;        // by degree
    std::vector<int64_t> loc_off, sinv_off; // n_cells + 1
    std::vector<int32_t> loc2glob;
    std::vector<int32_t> inc_ptr, inc_idx;  // unknown -> local positions (CSR)
    std::vector<int32_t> order, item_start, item_count, item_p;
    std::vector<int32_t> cclass;            // C_K class of each cell
    std::vector<int64_t> c_off;             // offset of each class in C
    std::vector<double> C;
    std::vector<int32_t> vert;              // interior-vertex unknowns, tensor order
    int nv[3] = {1, 1, 1};                  // interior vertices per direction
    std::vector<int32_t> ent_first, ent_n;  // other entities: first unknown, count
    std::vector<int64_t> ent_off;           // offset of the entity's inverse in inv
    std::vector<double> inv;                // inverses of A restricted to an entity
    // chunks of entities sharing one inverse (dev::hp_ent_cap per chunk), the
    // largest entities first: entity numbers chunk by chunk, each chunk's
    // first position and count, and the LDS elements of the largest chunk
    std::vector<int32_t> ent_list, ent_cstart, ent_ccount;
    int ent_lds = 0;
};

// lds_elems: LDS elements per buffer of the cell kernels (bounds cells per item)
void hp_build_host(const Mesh& M, int lds_elems, HpHost& H);
// the work items over H.order: runs of equal-degree cells whose local
// coefficients total at most min(lds_elems, item_elems) (at least one cell)
void hp_make_items(const Mesh& M, int lds_elems, int item_elems, HpHost& H);

}  // namespace hpg
