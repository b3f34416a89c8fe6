// Internal declarations shared by the host-side translation units of the
// hierarchical-matrix engine.  Not part of the ABI.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/hm.h"

namespace hm {

void set_error(const std::string& msg);

struct Layout {
    int64_t n = 0;
    int32_t leaf_size = 64;
    double eta = 2.0;
    int32_t partition = 0;   // HM_PART_*
    int32_t blr_depth = 0;   // balanced trees: level of every leaf
    int32_t depth = 0;
    std::vector<int64_t> perm;
    // nodes, depth-first pre-order
    std::vector<int64_t> node_begin, node_end;
    std::vector<int32_t> node_level, node_parent, node_son0, node_son1;
    std::vector<double> node_lo, node_hi;   // 3 per node
    // block-tree leaves, depth-first order
    std::vector<int32_t> blk_tau, blk_sigma, blk_adm;

    int64_t size(int32_t v) const { return node_end[v] - node_begin[v]; }
    bool leaf(int32_t v) const { return node_son0[v] < 0; }
};

// Storage rounding shared by hm_upload and hm_round_host.
double round_to(int32_t dtype, double v);
double dtype_max(int32_t dtype);
int dtype_bytes(int32_t dtype);
// encode a value that is already representable in dtype into its bit pattern
uint64_t encode(int32_t dtype, double v);

// Codecs of Sec. 4.1 (FPX rows, AFLP)
bool is_fpx(int32_t dt);
bool is_aflp(int32_t dt);
int aflp_width(int32_t dt);                 // bytes of an AFLP dtype
int32_t aflp_dtype(int bytes);
bool storage_dtype(int32_t dt);             // a format values can be stored in
int m_eps(double eps);                      // ceil(-log2 eps)
int32_t fpx_for_eps(double eps);            // FPX row (as a dtype) for accuracy eps
int aflp_scale_exp(const double* col, int64_t m);      // k of the column scale 2^k
int aflp_column_ebits(const double* col, int64_t m);   // exponent bits of one column
int aflp_matrix_ebits(const double* A, int64_t m, int64_t k);
bool aflp_feasible(int bytes, int e);
int aflp_direct_width(int e, double eps);   // bytes for direct compression (0: FP64)
// code word of v (scale 2^k, exponent width e, B bytes); *value = the stored value
uint64_t aflp_encode(double v, int k, int e, int bytes, double* value);

}  // namespace hm

struct hm_layout {
    hm::Layout L;
};
