// Reference-element tables for the DG discretisation, computed on the host in
// FP64.  Modal orthonormal bases: normalised Legendre polynomials on [-1, 1]
// (paper Sec. 5) and the Dubiner basis on the unit triangle; Gauss-Legendre
// rules on lines/edges and symmetric triangle rules with 3, 7 and 12 points.
#pragma once
#include <vector>

namespace bsw {

struct RefElement {
  int dim = 0, P = 0;
  int np = 0;   // basis functions
  int nq = 0;   // volume quadrature points
  int nfq = 0;  // points per face
  int nfc = 0;  // faces per element
  int nf = 0;   // fields
  std::vector<double> qxi;   // [nq][2] reference coordinates
  std::vector<double> qw;    // [nq] weights (sum = reference measure)
  std::vector<double> phi;   // [nq][np]
  std::vector<double> dphi;  // [nq][np][2] reference gradient
  std::vector<double> fphi;  // [nfc][nfq][np]
  std::vector<double> fw;    // [nfq] weights on [-1, 1]
  double measure = 0.0;
};

// Returns false for unsupported (dim, P).
bool build_reference(int dim, int P, RefElement& out);

// Basis values (and reference gradients) at arbitrary reference points.
void eval_basis(int dim, int P, double xi, double eta, double* phi, double* dphi /*[np][2] or null*/);

}  // namespace bsw
