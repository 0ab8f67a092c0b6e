// Presolve and postsolve of Section 4.5 (host code of libabip).
//
// The input is the bounded LP  min c^T x  s.t.  A x = b,  l <= x <= w  with a
// dense row-major A on the host; the output is the standard form
// min c~^T x~  s.t.  A~ x~ = b~,  x~ >= 0  that abip_setup takes, and a record
// that maps a solution of it back (postsolve).
//
// Reductions in the order of the paper's list, repeated until none applies,
// each scan in ascending index order (so the result is unique):
//   P3 l_j > w_j: infeasible.
//   P4 l_j = w_j: x_j fixed, substituted out of b.
//   P1 an empty row: dropped when |b_i| <= 1e-9 (1 + max|b|), else infeasible.
//   P2 an empty column: x_j at the bound its cost favours (lower for c_j > 0,
//      upper for c_j < 0, for c_j = 0 the finite one, lower first, else 0);
//      a favoured bound at infinity: unbounded.
//   P6 a singleton row a_ik x_k = b_i fixes x_k = b_i / a_ik (infeasible when
//      outside [l_k, w_k] by more than 1e-9 (1 + |bound|)); row and column leave.
// Then on the remaining columns: a free variable is split into x+ - x- (P5), one
// bounded only above is reflected (x = w - x'), the rest are shifted
// (x = l + x~), and every finite upper bound becomes a row x~_j + t_j = w_j - l_j
// with a slack column.  Dependent rows are kept (P7 is not applied): the method's
// linear step uses I + A A^T, nonsingular for any A.
//
// Postsolve: x from the reduced solution and the fixed values; y of kept rows
// from the reduced multipliers, 0 for empty rows, and for each singleton row (in
// reverse order of removal) the value that zeroes the reduced cost of the
// variable it fixed; r = c - A^T y.
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

#include "abip.h"

int abip_internal_fail(int code, const char* fmt, ...);

struct abip_presolve_t {
    int32_t m = 0, n = 0;
    std::vector<double> A, b, c;            // original data (A row-major)
    std::vector<int32_t> rows, cols;        // kept original rows / columns
    std::vector<int32_t> fixed_col;         // fixed columns, in fixing order
    std::vector<double> fixed_val;
    std::vector<int32_t> rm_kind, rm_row, rm_col;   // removed rows: 0 empty, 1 singleton
    // per kept column: kind (0 shift, 1 reflect, 2 free), first and second
    // standard column, bounds
    std::vector<int32_t> ck, cp, cq;
    std::vector<double> cl, cw;
    int32_t m_std = 0, n_std = 0;
    std::vector<double> As, bs, cs;         // the standard form (As row-major m_std x n_std)
    double obj_offset = 0.0;
    int32_t status = 0;                     // ABIP_PRESOLVE_*
    int32_t where = -1;                     // the row / column that decided a verdict
};

extern "C" int abip_presolve(int32_t m, int32_t n, const double* A, const double* b, const double* c,
                             const double* l, const double* w, abip_presolve_t** out, int32_t* status,
                             int32_t* m_std, int32_t* n_std) {
    if (!out) return abip_internal_fail(ABIP_E_INVALID, "abip_presolve: null output");
    *out = nullptr;
    if (m < 0 || n < 1) return abip_internal_fail(ABIP_E_DIM, "abip_presolve: bad dimensions m=%d n=%d", m, n);
    if ((m > 0 && (!A || !b)) || !c) return abip_internal_fail(ABIP_E_INVALID, "abip_presolve: null A, b or c");
    for (int64_t e = 0; e < (int64_t)m * n; ++e)
        if (!std::isfinite(A[e])) return abip_internal_fail(ABIP_E_NONFINITE, "abip_presolve: A has a non-finite entry");
    for (int i = 0; i < m; ++i)
        if (!std::isfinite(b[i])) return abip_internal_fail(ABIP_E_NONFINITE, "abip_presolve: b has a non-finite entry");
    for (int j = 0; j < n; ++j) {
        if (!std::isfinite(c[j])) return abip_internal_fail(ABIP_E_NONFINITE, "abip_presolve: c has a non-finite entry");
        if ((l && (std::isnan(l[j]) || l[j] == INFINITY)) || (w && (std::isnan(w[j]) || w[j] == -INFINITY)))
            return abip_internal_fail(ABIP_E_INVALID, "abip_presolve: bound of column %d is NaN or on the wrong side", j);
    }
    abip_presolve_t* p = new (std::nothrow) abip_presolve_t();
    if (!p) return abip_internal_fail(ABIP_E_OOM, "abip_presolve: out of host memory");
    p->m = m; p->n = n;
    p->A.assign(A, A + (size_t)m * n);
    p->b.assign(b, b + m);
    p->c.assign(c, c + n);
    std::vector<double> lb(n, 0.0), ub(n, INFINITY), bw(p->b);
    if (l) lb.assign(l, l + n);
    if (w) ub.assign(w, w + n);
    std::vector<char> ralive(m, 1), calive(n, 1);
    double bmax = 0.0;
    for (int i = 0; i < m; ++i) bmax = std::fmax(bmax, std::fabs(p->b[i]));
    const double btol = 1e-9 * (1.0 + bmax);
    const double* a = p->A.data();
    auto fix = [&](int j, double v) {
        for (int i = 0; i < m; ++i)
            if (ralive[i] && a[(size_t)i * n + j] != 0.0) bw[i] -= a[(size_t)i * n + j] * v;
        p->obj_offset += p->c[j] * v;
        p->fixed_col.push_back(j);
        p->fixed_val.push_back(v);
        calive[j] = 0;
    };
    auto verdict = [&](int st, int at) {
        p->status = st;
        p->where = at;
        *out = p;
        if (status) *status = st;
        if (m_std) *m_std = 0;
        if (n_std) *n_std = 0;
        return ABIP_OK;
    };
    bool changed = true;
    while (changed) {
        changed = false;
        for (int j = 0; j < n; ++j)                                    // P3
            if (calive[j] && lb[j] > ub[j]) return verdict(ABIP_PRESOLVE_INFEASIBLE, j);
        for (int j = 0; j < n; ++j)                                    // P4
            if (calive[j] && lb[j] == ub[j]) { fix(j, lb[j]); changed = true; }
        for (int i = 0; i < m; ++i) {                                  // P1
            if (!ralive[i]) continue;
            bool empty = true;
            for (int j = 0; j < n && empty; ++j) empty = !(calive[j] && a[(size_t)i * n + j] != 0.0);
            if (!empty) continue;
            if (std::fabs(bw[i]) > btol) return verdict(ABIP_PRESOLVE_INFEASIBLE, i);
            ralive[i] = 0;
            p->rm_kind.push_back(0); p->rm_row.push_back(i); p->rm_col.push_back(-1);
            changed = true;
        }
        for (int j = 0; j < n; ++j) {                                  // P2
            if (!calive[j]) continue;
            bool empty = true;
            for (int i = 0; i < m && empty; ++i) empty = !(ralive[i] && a[(size_t)i * n + j] != 0.0);
            if (!empty) continue;
            double v;
            if (p->c[j] > 0.0) {
                if (!std::isfinite(lb[j])) return verdict(ABIP_PRESOLVE_UNBOUNDED, j);
                v = lb[j];
            } else if (p->c[j] < 0.0) {
                if (!std::isfinite(ub[j])) return verdict(ABIP_PRESOLVE_UNBOUNDED, j);
                v = ub[j];
            } else {
                v = std::isfinite(lb[j]) ? lb[j] : (std::isfinite(ub[j]) ? ub[j] : 0.0);
            }
            fix(j, v);
            changed = true;
        }
        for (int i = 0; i < m; ++i) {                                  // P6
            if (!ralive[i]) continue;
            int cnt = 0, k = -1;
            for (int j = 0; j < n && cnt < 2; ++j)
                if (calive[j] && a[(size_t)i * n + j] != 0.0) { ++cnt; k = j; }
            if (cnt != 1) continue;
            const double v = bw[i] / a[(size_t)i * n + k];
            if (v < lb[k] - 1e-9 * (1.0 + std::fabs(lb[k])) || v > ub[k] + 1e-9 * (1.0 + std::fabs(ub[k])))
                return verdict(ABIP_PRESOLVE_INFEASIBLE, i);
            ralive[i] = 0;
            p->rm_kind.push_back(1); p->rm_row.push_back(i); p->rm_col.push_back(k);
            fix(k, v);
            changed = true;
        }
    }
    for (int i = 0; i < m; ++i) if (ralive[i]) p->rows.push_back(i);
    for (int j = 0; j < n; ++j) if (calive[j]) p->cols.push_back(j);
    // reformulation: standard columns (sign, original column), upper-bound rows
    std::vector<double> sgn;
    std::vector<int32_t> src;
    std::vector<int32_t> ubp;
    std::vector<double> ubv;
    for (int32_t j : p->cols) {
        const double lj = lb[j], wj = ub[j];
        const int pcol = (int)src.size();
        if (!std::isfinite(lj) && !std::isfinite(wj)) {
            sgn.push_back(1.0); src.push_back(j);
            sgn.push_back(-1.0); src.push_back(j);
            p->ck.push_back(2); p->cp.push_back(pcol); p->cq.push_back(pcol + 1);
        } else if (!std::isfinite(lj)) {
            sgn.push_back(-1.0); src.push_back(j);
            p->ck.push_back(1); p->cp.push_back(pcol); p->cq.push_back(-1);
        } else {
            sgn.push_back(1.0); src.push_back(j);
            p->ck.push_back(0); p->cp.push_back(pcol); p->cq.push_back(-1);
            if (std::isfinite(wj)) { ubp.push_back(pcol); ubv.push_back(wj - lj); }
        }
        p->cl.push_back(lj); p->cw.push_back(wj);
    }
    const int mk = (int)p->rows.size(), nk = (int)src.size(), nu = (int)ubp.size();
    p->m_std = mk + nu;
    p->n_std = nk + nu;
    p->As.assign((size_t)p->m_std * p->n_std, 0.0);
    p->bs.assign(p->m_std, 0.0);
    p->cs.assign(p->n_std, 0.0);
    for (int r = 0; r < mk; ++r) p->bs[r] = bw[p->rows[r]];
    for (int q = 0; q < nk; ++q) {
        const int j = src[q];
        for (int r = 0; r < mk; ++r) p->As[(size_t)r * p->n_std + q] = sgn[q] * a[(size_t)p->rows[r] * n + j];
        p->cs[q] = sgn[q] * p->c[j];
    }
    // constants of the shift (x = l + x~) and the reflection (x = w - x')
    for (size_t t = 0; t < p->cols.size(); ++t) {
        if (p->ck[t] == 2) continue;
        const int j = p->cols[t];
        const double x0 = (p->ck[t] == 0) ? p->cl[t] : p->cw[t];
        if (x0 == 0.0) continue;
        for (int r = 0; r < mk; ++r) {
            const double aij = a[(size_t)p->rows[r] * n + j];
            if (aij != 0.0) p->bs[r] -= aij * x0;
        }
        p->obj_offset += p->c[j] * x0;
    }
    for (int t = 0; t < nu; ++t) {
        p->As[(size_t)(mk + t) * p->n_std + ubp[t]] = 1.0;
        p->As[(size_t)(mk + t) * p->n_std + nk + t] = 1.0;
        p->bs[mk + t] = ubv[t];
    }
    p->status = ABIP_PRESOLVE_REDUCED;
    *out = p;
    if (status) *status = p->status;
    if (m_std) *m_std = p->m_std;
    if (n_std) *n_std = p->n_std;
    return ABIP_OK;
}

extern "C" int abip_presolve_get(const abip_presolve_t* p, double* A_std, double* b_std, double* c_std,
                                 double* obj_offset) {
    if (!p) return abip_internal_fail(ABIP_E_INVALID, "abip_presolve_get: null record");
    if (p->status != ABIP_PRESOLVE_REDUCED)
        return abip_internal_fail(ABIP_E_STATE, "abip_presolve_get: the presolve ended with a verdict (%d)", p->status);
    if (A_std) std::memcpy(A_std, p->As.data(), sizeof(double) * p->As.size());
    if (b_std) std::memcpy(b_std, p->bs.data(), sizeof(double) * p->bs.size());
    if (c_std) std::memcpy(c_std, p->cs.data(), sizeof(double) * p->cs.size());
    if (obj_offset) *obj_offset = p->obj_offset;
    return ABIP_OK;
}

extern "C" int abip_presolve_info(const abip_presolve_t* p, int32_t* where, int32_t* rows_kept, int32_t* cols_kept,
                                  int32_t* row_kind, int32_t* fixed_cols, double* fixed_vals, int32_t* nfixed) {
    if (!p) return abip_internal_fail(ABIP_E_INVALID, "abip_presolve_info: null record");
    if (where) *where = p->where;
    if (rows_kept) std::memcpy(rows_kept, p->rows.data(), sizeof(int32_t) * p->rows.size());
    if (cols_kept) std::memcpy(cols_kept, p->cols.data(), sizeof(int32_t) * p->cols.size());
    if (row_kind) {
        for (int i = 0; i < p->m; ++i) row_kind[i] = -1;
        for (size_t t = 0; t < p->rm_row.size(); ++t) row_kind[p->rm_row[t]] = p->rm_kind[t];
    }
    if (fixed_cols) std::memcpy(fixed_cols, p->fixed_col.data(), sizeof(int32_t) * p->fixed_col.size());
    if (fixed_vals) std::memcpy(fixed_vals, p->fixed_val.data(), sizeof(double) * p->fixed_val.size());
    if (nfixed) *nfixed = (int32_t)p->fixed_col.size();
    return ABIP_OK;
}

extern "C" int abip_postsolve(const abip_presolve_t* p, const double* x_std, const double* y_std, double* x,
                              double* y, double* r) {
    if (!p) return abip_internal_fail(ABIP_E_INVALID, "abip_postsolve: null record");
    if (p->status != ABIP_PRESOLVE_REDUCED)
        return abip_internal_fail(ABIP_E_STATE, "abip_postsolve: the presolve ended with a verdict (%d)", p->status);
    if (!x_std || !y_std || !x || !y || !r) return abip_internal_fail(ABIP_E_INVALID, "abip_postsolve: null vector");
    const int m = p->m, n = p->n;
    const double* a = p->A.data();
    for (int j = 0; j < n; ++j) x[j] = 0.0;
    for (size_t t = 0; t < p->fixed_col.size(); ++t) x[p->fixed_col[t]] = p->fixed_val[t];
    for (size_t t = 0; t < p->cols.size(); ++t) {
        const int j = p->cols[t];
        if (p->ck[t] == 2) x[j] = x_std[p->cp[t]] - x_std[p->cq[t]];
        else if (p->ck[t] == 1) x[j] = p->cw[t] - x_std[p->cp[t]];
        else x[j] = p->cl[t] + x_std[p->cp[t]];
    }
    for (int i = 0; i < m; ++i) y[i] = 0.0;
    for (size_t t = 0; t < p->rows.size(); ++t) y[p->rows[t]] = y_std[t];
    for (size_t t = p->rm_row.size(); t-- > 0;) {
        if (p->rm_kind[t] != 1) continue;
        const int i = p->rm_row[t], k = p->rm_col[t];
        double rest = 0.0;
        for (int q = 0; q < m; ++q)
            if (q != i) rest += a[(size_t)q * n + k] * y[q];
        y[i] = (p->c[k] - rest) / a[(size_t)i * n + k];
    }
    for (int j = 0; j < n; ++j) {
        double s = 0.0;
        for (int i = 0; i < m; ++i) s += a[(size_t)i * n + j] * y[i];
        r[j] = p->c[j] - s;
    }
    return ABIP_OK;
}

extern "C" int abip_presolve_free(abip_presolve_t* p) {
    delete p;
    return ABIP_OK;
}
