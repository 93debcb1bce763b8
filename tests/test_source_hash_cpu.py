"""The kernel-source hash that ties counter summaries to the code they were
taken on: comments and layout do not change it, code does."""
from paper_2112_06396_amd import build


def test_comments_and_layout_are_ignored():
    a = "int f(int x) {  // twice x\n    return 2 * x; /* doubled\n  here */ }\n"
    b = "int f(int x) {\n  return 2 * x;\n}\n// a note\n"
    assert build._code_only(a) == build._code_only(b) == "int f(int x) { return 2 * x; }"


def test_code_changes_are_not_ignored():
    a = "int f(int x) { return 2 * x; }"
    assert build._code_only(a) != build._code_only(a.replace("2 *", "3 *"))
    assert build._code_only("a/b") == "a/b"  # a division is not a comment


def test_source_hash_is_stable():
    h = build.source_hash()
    assert len(h) == 16 and h == build.source_hash()
