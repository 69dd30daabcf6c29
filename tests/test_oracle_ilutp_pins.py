"""Hand-worked pins for the oracle's ILUTP rules that bind only in special
situations (Section 3.2 eq. (ilu); Section 4's settings): the pivot threshold
permtol on either side of the diagonal-to-largest ratio, the fill limit of
nL0 + p multipliers and nU0 + p off-diagonal U entries with its tie-break, and
the relative drop tolerance.  Every expected value below is worked out by hand
in the comments from the row algorithm (Saad's ILUTP, which Section 4 names):
no expected value comes from running the oracle."""
import pytest

from oracle.ilutp import ilutp, paper_lfil


def _rows(dense):
    return [{j: float(v) for j, v in enumerate(r) if v != 0.0} for r in dense]


# Row 0 is (0.07, 1.0, 0): its diagonal is 0.07 of its largest entry.
A3 = [[0.07, 1.0, 0.0],
      [0.5, 0.2, 0.3],
      [0.0, 0.4, 1.0]]


def test_pivot_swaps_when_permtol_times_max_exceeds_diagonal():
    # permtol 0.1: 0.1 * 1.0 = 0.1 > 0.07, so columns 0 and 1 swap at row 0:
    # q = (1, 0, 2) and u_00 = 1.0, u_01 = 0.07.
    # Row 1, original (0.5, 0.2, 0.3): column 1 sits at position 0, so
    # l_10 = 0.2 / 1.0 = 0.2; column 0 (position 1) becomes 0.5 - 0.2 * 0.07
    # = 0.486, column 2 stays 0.3; the diagonal 0.486 is the largest: no swap.
    # Row 2, original (0, 0.4, 1.0): l_20 = 0.4; fill at column 0:
    # 0 - 0.4 * 0.07 = -0.028 (position 1), so l_21 = -0.028 / 0.486 and
    # u_22 = 1.0 - l_21 * 0.3.
    L, U, q = ilutp(_rows(A3), 3, droptol=0.0, permtol=0.1, lfil=3)
    assert list(q) == [1, 0, 2]
    assert U[0] == pytest.approx({0: 1.0, 1: 0.07}, abs=0, rel=1e-15)
    assert L[1] == pytest.approx({0: 0.2}, rel=1e-15)
    assert U[1] == pytest.approx({1: 0.486, 2: 0.3}, rel=1e-14)
    l21 = -0.028 / 0.486
    assert L[2] == pytest.approx({0: 0.4, 1: l21}, rel=1e-14)
    assert U[2] == pytest.approx({2: 1.0 - l21 * 0.3}, rel=1e-14)


def test_pivot_keeps_diagonal_when_permtol_times_max_is_below_it():
    # permtol 0.05: 0.05 * 1.0 = 0.05 < 0.07, no swap: q = identity,
    # u_00 = 0.07, u_01 = 1.0.  Row 1: l_10 = 0.5 / 0.07; column 1 becomes
    # 0.2 - l_10 * 1.0 = -6.942857...; it is the row's largest: no swap.
    # Row 2: only column 1 (position 1) is left of the diagonal:
    # l_21 = 0.4 / u_11, u_22 = 1.0 - l_21 * 0.3.
    L, U, q = ilutp(_rows(A3), 3, droptol=0.0, permtol=0.05, lfil=3)
    assert list(q) == [0, 1, 2]
    l10 = 0.5 / 0.07
    u11 = 0.2 - l10 * 1.0
    assert U[0] == pytest.approx({0: 0.07, 1: 1.0}, rel=1e-15)
    assert L[1] == pytest.approx({0: l10}, rel=1e-15)
    assert U[1] == pytest.approx({1: u11, 2: 0.3}, rel=1e-14)
    assert L[2] == pytest.approx({1: 0.4 / u11}, rel=1e-14)
    assert U[2] == pytest.approx({2: 1.0 - (0.4 / u11) * 0.3}, rel=1e-14)


def test_pivot_takes_largest_entry_of_the_whole_row():
    # Row 0 = (0.01, 0.5, 2.0): with permtol 0.1 the swap goes to column 2,
    # the largest of the row, not to the first entry above the threshold.
    A = [[0.01, 0.5, 2.0], [1.0, 1.0, 0.0], [0.0, 1.0, 1.0]]
    L, U, q = ilutp(_rows(A), 3, droptol=0.0, permtol=0.1, lfil=3)
    assert q[0] == 2
    assert U[0][0] == 2.0


# Fill limit.  Row 2 = (1, 0, 5, 0) has one original entry left of the
# diagonal (nL0 = 1) and none right of it (nU0 = 0); with p = 0 it keeps one
# multiplier and no off-diagonal U entry.
#   row 0 = (2, 2, 0, 1): u_00 = 2, u_01 = 2, u_03 = 1
#   row 1 = (0, 2, 0, 0): u_11 = 2
#   row 2: l_20 = 1/2 = 0.5; fill at column 1: 0 - 0.5*2 = -1 and column 3:
#          0 - 0.5*1 = -0.5; then l_21 = -1/2 = -0.5: two multipliers of equal
#          magnitude 0.5, and the tie goes to the lower position, so only l_20
#          is kept; the U fill -0.5 at column 3 exceeds nU0 + p = 0 and goes.
A4 = [[2.0, 2.0, 0.0, 1.0],
      [0.0, 2.0, 0.0, 0.0],
      [1.0, 0.0, 5.0, 0.0],
      [0.0, 0.0, 0.0, 3.0]]


def test_fill_limit_keeps_original_count_plus_p_with_ties_to_lower_position():
    L, U, q = ilutp(_rows(A4), 4, droptol=0.0, permtol=0.0, lfil=0)
    assert list(q) == [0, 1, 2, 3]
    assert L[2] == {0: 0.5}
    assert U[2] == {2: 5.0}
    assert U[0] == {0: 2.0, 1: 2.0, 3: 1.0}


def test_fill_limit_keeps_the_largest_multiplier():
    # Row 0 = (2, 1, 0, 0), row 1 = (0, 4, 0, 0), row 2 = (1, 0, 5, 0):
    # l_20 = 0.5, the fill at column 1 is 0 - 0.5 * 1 = -0.5, so
    # l_21 = -0.5 / 4 = -0.125.  nL0 = 1 and p = 0: only the larger, l_20, stays.
    A = [[2.0, 1.0, 0.0, 0.0], [0.0, 4.0, 0.0, 0.0], [1.0, 0.0, 5.0, 0.0], [0.0, 0.0, 0.0, 1.0]]
    L, U, q = ilutp(_rows(A), 4, droptol=0.0, permtol=0.0, lfil=0)
    assert L[2] == {0: 0.5}
    L, U, q = ilutp(_rows(A), 4, droptol=0.0, permtol=0.0, lfil=1)
    assert L[2] == {0: 0.5, 1: -0.125}


def test_fill_limit_with_p_one_keeps_both_multipliers_and_the_fill():
    # p = 1: room for 1 + 1 multipliers and 0 + 1 off-diagonal U entries;
    # both multipliers stay (0.5 and -0.5); the eliminated column 1 no longer
    # updates anything (row 1 has only its diagonal), so u_23 = -0.5.
    L, U, q = ilutp(_rows(A4), 4, droptol=0.0, permtol=0.0, lfil=1)
    assert L[2] == {0: 0.5, 1: -0.5}
    assert U[2] == {2: 5.0, 3: -0.5}


def test_fill_limit_keeps_the_largest_not_the_first():
    # Row 0 = (1, 0, 0, 0, 0, -2.5), the other rows identity except row 2 =
    # (1, 0, 4, 1, 3, 0).  Row 2: l_20 = 1; the fill at column 5 is
    # 0 - 1 * (-2.5) = 2.5, so its U part is {3: 1, 4: 3, 5: 2.5} besides the
    # diagonal.  nU0 = 2 (columns 3 and 4 are nonzero in A) and p = 0: the two
    # largest stay, 3 and the fill 2.5; the original entry 1 at column 3 goes.
    A = [[1.0, 0.0, 0.0, 0.0, 0.0, -2.5],
         [0.0, 1.0, 0.0, 0.0, 0.0, 0.0],
         [1.0, 0.0, 4.0, 1.0, 3.0, 0.0],
         [0.0, 0.0, 0.0, 1.0, 0.0, 0.0],
         [0.0, 0.0, 0.0, 0.0, 1.0, 0.0],
         [0.0, 0.0, 0.0, 0.0, 0.0, 1.0]]
    L, U, q = ilutp(_rows(A), 6, droptol=0.0, permtol=0.0, lfil=0)
    assert L[2] == {0: 1.0}
    assert U[2] == {2: 4.0, 4: 3.0, 5: 2.5}


def test_drop_tolerance_relative_to_the_row_two_norm():
    # Row 1 = (0.3, 4, 0, 0.04): ||a_1||_2 = sqrt(0.09 + 16 + 0.0016) =
    # 4.01140..., so droptol 0.01 gives tau = 0.0401140: the entry 0.04 at
    # column 3 is dropped (0.04 < tau) while l_10 = 0.3 / 2 = 0.15 stays; the
    # fill 0 - 0.15 * 0.5 = -0.075 at column 2 stays (0.075 >= tau).
    A = [[2.0, 0.0, 0.5, 0.0],
         [0.3, 4.0, 0.0, 0.04],
         [0.0, 0.0, 1.0, 0.0],
         [0.0, 0.0, 0.0, 1.0]]
    L, U, q = ilutp(_rows(A), 4, droptol=0.01, permtol=0.0, lfil=4)
    assert L[1] == pytest.approx({0: 0.15}, rel=1e-15)
    assert U[1] == pytest.approx({1: 4.0, 2: -0.075}, rel=1e-15)
    # droptol 0.009: tau = 0.0361..., so 0.04 is kept
    L, U, q = ilutp(_rows(A), 4, droptol=0.009, permtol=0.0, lfil=4)
    assert U[1] == pytest.approx({1: 4.0, 2: -0.075, 3: 0.04}, rel=1e-15)


def test_paper_fill_rule():
    # Section 4: extra fill of half the average number of nonzeros per row,
    # rounded up: 85 nonzeros over 10 rows -> ceil(4.25) = 5; 84 -> 5; 80 -> 4.
    assert paper_lfil(85, 10) == 5
    assert paper_lfil(84, 10) == 5
    assert paper_lfil(80, 10) == 4
