// Host preprocessing declarations (validation, preconditioning, transpose, schedules).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "hprlp_internal.h"

namespace hprlp {

struct Scaling {
    std::vector<double> val;  // A~ = D_r A D_c, CSR order of A
    std::vector<double> dr, dc;
};

int validate_problem(int64_t m1, int64_t m2, int64_t n, const int64_t *rowptr,
                     const int32_t *colidx, const double *val, const double *b,
                     const double *c, const double *l, const double *u,
                     const hprlp_options &o, std::string &err);
int validate_options(const hprlp_options &o, std::string &err);
void resolve_options(hprlp_options &o);
void transpose(int64_t m, int64_t n, const int64_t *rowptr, const int32_t *colidx,
               std::vector<int64_t> &rowptr_t, std::vector<int32_t> &colidx_t,
               std::vector<int32_t> &pos);
void precondition(int64_t m, int64_t n, const int64_t *rowptr, const int32_t *colidx,
                  const std::vector<int64_t> &rowptr_t, const std::vector<int32_t> &pos,
                  const double *val, const hprlp_options &o, Scaling &s);

}  // namespace hprlp
