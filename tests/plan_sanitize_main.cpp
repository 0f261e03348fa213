// Test driver: the host part of plan creation (system checks, screening, canonical pairs,
// every task list, workspace chunks, mixed-precision lists) built on its own with
// AddressSanitizer and UndefinedBehaviorSanitizer, in the order the library runs it.
//
// Input (binary, native byte order): int32 n_atoms, n_species, n_systems, periodic;
// double r_cut; int64 budget; int32 species[n_atoms]; double positions[3 n_atoms];
// int32 n_basis[n_species], n_aux[n_species]; int32 sys_atom_off[n_systems + 1];
// double lattice[9] if periodic.  Output: one line "n_pairs n_chunks intermediate_bytes".
#include "exx_internal.h"

#include <cstdio>
#include <vector>

template <typename T>
static bool get(FILE* f, T* x, size_t n) {
  return std::fread(x, sizeof(T), n, f) == n;
}

int main(int argc, char** argv) {
  if (argc != 2) return 64;
  FILE* f = std::fopen(argv[1], "rb");
  if (!f) return 65;
  int32_t head[4];
  double r_cut;
  int64_t budget;
  if (!get(f, head, 4) || !get(f, &r_cut, 1) || !get(f, &budget, 1)) return 66;
  const int na = head[0], ns = head[1], nsys = head[2], periodic = head[3];
  std::vector<int32_t> species(na), nb(ns), nx(ns), off(nsys + 1);
  std::vector<double> pos(3 * (size_t)na), lat(9);
  if (!get(f, species.data(), na) || !get(f, pos.data(), pos.size()) || !get(f, nb.data(), ns) ||
      !get(f, nx.data(), ns) || !get(f, off.data(), nsys + 1))
    return 66;
  if (periodic && !get(f, lat.data(), 9)) return 66;
  std::fclose(f);
  exx::HostPlan hp;
  std::string err;
  int rc = exx::describe_system(na, ns, species.data(), pos.data(), nb.data(), nx.data(), r_cut, nsys,
                                nsys > 1 ? off.data() : nullptr, periodic ? lat.data() : nullptr, hp, err);
  if (rc != 0) {
    std::fprintf(stderr, "describe_system: %s\n", err.c_str());
    return 2;
  }
  if (hp.periodic) exx::host_neighbors_periodic(hp);
  else exx::host_neighbors(hp);
  rc = hp.periodic ? exx::derive_lists_periodic(hp, err) : exx::derive_lists(hp, err);
  if (rc != 0) {
    std::fprintf(stderr, "lists: %s\n", err.c_str());
    return 3;
  }
  rc = exx::derive_chunks(hp, budget, err);
  if (rc != 0) {
    std::fprintf(stderr, "chunks: %s\n", err.c_str());
    return 4;
  }
  exx::derive_mixed_lists(hp, 0);
  exx::derive_mixed_lists(hp, 1);
  std::printf("%zu %zu %lld\n", hp.pair_a.size(), hp.chunks.empty() ? (size_t)1 : hp.chunks.size(),
              (long long)(8 * hp.ws_total));
  return 0;
}
